"""Seeded synthetic inputs and workload descriptions.

This module is shared by the FP64 oracle's tests, the GPU parity tests and the
benchmark.  It holds no arithmetic of the method: only the workload shapes, the
parameter values the paper prints, and seeded random draws (white noise,
momenta, the cheap count recipe used for timing runs).

Workloads (all distances in Mpc/h):
  c0    32^3,  L=250,  Phi-web, 4 regions, mean count 0.5, NB beta 5
  c0fd  16^3,  L=125,  same model (finite-difference size)
  c1    128^3, L=500,  Phi-web, 4 regions, mean count 1.0, NB beta 5
  c2    256^3, L=1000, Phi-web (R=8) x delta-web (R=2), 16 regions, plane-parallel
        RSD along z, mean count 2.0, NB beta 3
  c3    32 chains: 12 x 64^3 (L=256), 10 x 96^3 (L=384), 10 x 128^3 (L=512)
  c4    512^3, L=2000, as c2, 20-step leapfrog trajectory
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

WEB_PHI = 0     # tidal tensor of the potential, Phi = inverse Laplacian of delta
WEB_DELTA = 1   # Hessian of the (smoothed) density, scaled by ell^2, sign flipped

# Section 3, Table 'values', TEST1 row (voids, sheets, filaments, knots).
TEST1_ALPHA = (1.10, 1.03, 1.15, 1.23)
TEST1_BETA = (10.10, 13.70, 12.10, 14.40)
# Section 3, Table 'values', TEST2 row.
TEST2_ALPHA = (1.05, 1.11, 1.23, 1.30)
TEST2_BETA = (7.10, 8.70, 8.10, 9.40)
# Section 3, Table 'values3' (TEST3): rows Phi-class x delta-sub-class,
# columns (alpha, beta, epsilon, rho).
TEST3_TABLE = (
    (1.29, 5.80, 1.02, 0.22), (1.05, 14.30, 1.06, 0.26),
    (1.14, 11.87, 0.97, 0.16), (1.34, 10.60, 1.00, 0.20),
    (1.04, 10.74, 1.00, 0.20), (1.06, 11.57, 0.97, 0.17),
    (1.11, 12.59, 0.98, 0.18), (1.05, 13.67, 1.06, 0.26),
    (0.94, 5.71, 1.02, 0.22), (1.13, 13.42, 0.93, 0.13),
    (1.27, 7.75, 0.96, 0.16), (1.20, 11.21, 1.01, 0.21),
    (1.18, 8.36, 0.99, 0.19), (1.01, 11.24, 0.96, 0.16),
    (1.07, 10.99, 0.94, 0.14), (1.17, 9.71, 1.08, 0.28),
)
# Section 3: log-normal prior hyper-parameters for alpha and beta.
PRIOR_MU_ALPHA, PRIOR_SIGMA_ALPHA = 0.27, 0.30
PRIOR_MU_BETA, PRIOR_SIGMA_BETA = 2.12, 0.20

# Column order of a bias table row.
COL_ALPHA, COL_EPS, COL_RHO, COL_BETA = 0, 1, 2, 3


RSD_RADIAL = 3   # rsd_axis value: radial RSD about an observer at the box centre


@dataclass(frozen=True)
class Cosmo:
    """Fixed cosmology and gravity-solver settings (held fixed, Section 2.1)."""
    omega_m: float = 0.31
    h: float = 0.68
    sigma8: float = 0.81
    n_s: float = 0.96
    d1: float = 1.0            # linear growth at the output redshift (z=0)
    f_growth: float = 0.31 ** 0.55  # linear growth rate used by RSD
    r_s: float = 4.0           # ALPT Gaussian smoothing radius
    rsd_axis: int = -1         # -1: real space; 0..2: plane-parallel along that axis; 3: radial (RSD_RADIAL)
    tau_sc: float = 0.05       # width of the smooth spherical-collapse hinge (0 = exact max)
    x_floor: float = 1e-6      # floor on 1+delta inside the bias


@dataclass(frozen=True)
class Web:
    """Fuzzy cosmic-web settings (Section 2.8)."""
    kinds: Tuple[int, ...] = (WEB_PHI,)
    smooth_r: Tuple[float, ...] = (0.0,)
    ell: Tuple[float, ...] = (0.0,)
    steepness: float = 20.0
    lambda_th: float = 0.1

    @property
    def n_webs(self) -> int:
        return len(self.kinds)

    @property
    def n_regions(self) -> int:
        return 4 ** len(self.kinds)


@dataclass
class Chain:
    """One chain of a workload: its mesh, box, truth bias table and seeds."""
    n: int
    box: float
    bias: np.ndarray           # [R, 4] float64: alpha, eps, rho_th, beta
    mean_count: float
    seed_key: Tuple[int, int]  # (workload index, chain index)

    @property
    def dx(self) -> float:
        return self.box / self.n


@dataclass
class Workload:
    name: str
    index: int
    cosmo: Cosmo
    web: Web
    chains: List[Chain]
    leapfrog_steps: int = 0
    # host-side tying of free parameters: list of (region list, column) per
    # free parameter; entries not listed stay at their table value.
    free: List[Tuple[Tuple[int, ...], int]] = field(default_factory=list)

    @property
    def n_regions(self) -> int:
        return self.web.n_regions


def four_class_table(alpha=TEST1_ALPHA, eps=-1.0, rho=0.2, beta=5.0) -> np.ndarray:
    t = np.zeros((4, 4))
    t[:, COL_ALPHA] = alpha
    t[:, COL_EPS] = eps
    t[:, COL_RHO] = rho
    t[:, COL_BETA] = beta
    return t


def sixteen_region_table(alpha=TEST1_ALPHA, beta=3.0) -> np.ndarray:
    """Alpha per Phi-class broadcast over delta-sub-classes; epsilon and rho
    from Table values3 with epsilon negated (low-density cut-off)."""
    t = np.zeros((16, 4))
    for j in range(4):
        for k in range(4):
            r = 4 * j + k
            row = TEST3_TABLE[r]
            t[r, COL_ALPHA] = alpha[j]
            t[r, COL_EPS] = -row[2]
            t[r, COL_RHO] = row[3]
            t[r, COL_BETA] = beta
    return t


def _four_class_free():
    return [((r,), COL_ALPHA) for r in range(4)]


def full_table_free(n_regions: int):
    """Every entry of the table free: the 16-region model's 64 parameters
    (alpha, eps, rho_th and beta of every region)."""
    return [((r,), col) for r in range(n_regions) for col in range(4)]


def _sixteen_free():
    out = []
    for j in range(4):
        out.append((tuple(4 * j + k for k in range(4)), COL_ALPHA))
    for j in range(4):
        out.append((tuple(4 * j + k for k in range(4)), COL_BETA))
    return out


def workload(name: str) -> Workload:
    """The named synthetic workload."""
    phi1 = Web()
    hier = Web(kinds=(WEB_PHI, WEB_DELTA), smooth_r=(8.0, 2.0), ell=(0.0, 2.0))
    if name == "c0":
        return Workload("c0", 0, Cosmo(), phi1,
                        [Chain(32, 250.0, four_class_table(), 0.5, (0, 0))],
                        free=_four_class_free())
    if name == "c0fd":
        return Workload("c0fd", 5, Cosmo(), phi1,
                        [Chain(16, 125.0, four_class_table(), 0.5, (5, 0))],
                        free=_four_class_free())
    if name == "c1":
        return Workload("c1", 1, Cosmo(), phi1,
                        [Chain(128, 500.0, four_class_table(), 1.0, (1, 0))],
                        free=_four_class_free())
    if name == "c2":
        return Workload("c2", 2, Cosmo(rsd_axis=2), hier,
                        [Chain(256, 1000.0, sixteen_region_table(), 2.0, (2, 0))],
                        free=_sixteen_free())
    if name == "c2w1":
        return Workload("c2w1", 6, Cosmo(), phi1,
                        [Chain(256, 1000.0, four_class_table(), 1.0, (6, 0))],
                        free=_four_class_free())
    if name == "c3":
        rng = np.random.default_rng(np.random.SeedSequence([3, 999]))
        chains = []
        sizes = [64] * 12 + [96] * 10 + [128] * 10
        for c, n in enumerate(sizes):
            a = np.array(TEST1_ALPHA) * rng.uniform(0.8, 1.2, size=4)
            chains.append(Chain(n, 4.0 * n, four_class_table(alpha=a), 1.0, (3, c)))
        return Workload("c3", 3, Cosmo(), phi1, chains, leapfrog_steps=10,
                        free=_four_class_free())
    if name == "c4":
        return Workload("c4", 4, Cosmo(rsd_axis=2), hier,
                        [Chain(512, 2000.0, sixteen_region_table(), 2.0, (4, 0))],
                        leapfrog_steps=20, free=_sixteen_free())
    raise KeyError(name)


def small_variant(w: Workload, n: int, box: Optional[float] = None) -> Workload:
    """Same model as `w` on a smaller mesh at the same cell size (for tests)."""
    c0 = w.chains[0]
    b = box if box is not None else c0.dx * n
    ch = Chain(n, b, c0.bias.copy(), c0.mean_count, (w.index, 100 + n))
    return dataclasses.replace(w, chains=[ch])


# ---------------------------------------------------------------- seeded draws
ROLE_TRUTH_NU, ROLE_DATA, ROLE_EVAL_NU, ROLE_MOMENTUM, ROLE_MISC = 0, 1, 2, 3, 4
NEAR_KAPPA = 0.05


def rng_for(chain: Chain, role: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([*chain.seed_key, role]))


def white_noise(chain: Chain, role: int = ROLE_EVAL_NU, dtype=np.float64) -> np.ndarray:
    """i.i.d. standard normal field on the chain's mesh, C order [x][y][z]."""
    g = rng_for(chain, role)
    n = chain.n
    return g.standard_normal((n, n, n)).astype(dtype)


def near_truth_noise(chain: Chain, kappa: float = NEAR_KAPPA) -> np.ndarray:
    """A white-noise state near the truth, sqrt(1-kappa^2) nu_truth + kappa xi,
    standing in for a state a converged chain visits."""
    return (np.sqrt(1.0 - kappa * kappa) * white_noise(chain, ROLE_TRUTH_NU)
            + kappa * white_noise(chain, ROLE_EVAL_NU))


def gamma_poisson_counts(nbar: np.ndarray, beta: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """Draw n* ~ Poisson(lambda), lambda ~ Gamma(shape=beta, scale=nbar/beta)."""
    lam = rng.gamma(shape=beta, scale=np.maximum(nbar, 0.0) / beta)
    n = rng.poisson(lam)
    return np.minimum(n, 65535).astype(np.uint16)


def timing_counts(chain: Chain, smooth_cells: float = 1.5) -> np.ndarray:
    """Cheap synthetic counts for timing runs at large meshes.

    A log-normal field (unit-variance Gaussian noise smoothed over a few cells,
    exponentiated) sets a clustered mean with the chain's mean count; counts are
    Gamma-Poisson draws around it with the chain's NB dispersion.  It mimics the
    clustering and count distribution of the mock data without running the
    forward model.
    """
    g = rng_for(chain, ROLE_DATA)
    n = chain.n
    w = g.standard_normal((n, n, n)).astype(np.float32)
    k = np.fft.fftfreq(n).astype(np.float32)
    kz = np.fft.rfftfreq(n).astype(np.float32)
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + kz[None, None, :] ** 2
    filt = np.exp(-0.5 * k2 * (2 * np.pi * smooth_cells) ** 2).astype(np.float32)
    s = np.fft.irfftn(np.fft.rfftn(w) * filt, s=w.shape, axes=(0, 1, 2)).astype(np.float32)
    s /= s.std() + 1e-30
    lam = np.exp(s - 0.5)
    lam *= chain.mean_count / lam.mean()
    beta = float(chain.bias[0, COL_BETA])
    return gamma_poisson_counts(lam, np.full_like(lam, beta), g)


def tie_array(w: Workload) -> np.ndarray:
    """Free-parameter index of every bias-table entry ([R][4] flattened), -1
    for the entries held fixed: the layout the sampling call takes."""
    tie = -np.ones(w.n_regions * 4, dtype=np.int64)
    for f, (regions, col) in enumerate(w.free):
        for r in regions:
            tie[r * 4 + col] = f
    return tie


def prior_arrays(w: Workload):
    """Gaussian prior (mean, sigma) on the log of the magnitude of every free
    bias parameter: the alpha and beta priors of the paper's tests; eps and
    rho_th (free only in the full table) centred on the first chain's table
    with width 0.3."""
    mu, sig = [], []
    for regions, col in w.free:
        if col == COL_BETA:
            mu.append(PRIOR_MU_BETA), sig.append(PRIOR_SIGMA_BETA)
        elif col == COL_ALPHA:
            mu.append(PRIOR_MU_ALPHA), sig.append(PRIOR_SIGMA_ALPHA)
        else:
            mu.append(float(np.log(abs(w.chains[0].bias[regions[0], col])))), sig.append(0.3)
    return np.array(mu), np.array(sig)


def free_start(w: Workload, chain: Chain) -> np.ndarray:
    """Log of the magnitude of the free bias parameters of a chain (the
    sampled coordinates)."""
    return np.log(np.abs(np.array([chain.bias[r[0], c] for r, c in w.free])))


def free_signs(w: Workload, chain: Chain) -> np.ndarray:
    """Sign of every free bias parameter in a chain's table (+1 or -1)."""
    return np.where(np.array([chain.bias[r[0], c] for r, c in w.free]) < 0, -1, 1).astype(np.int64)


def bytes_model(n: int, n_webs: int, leapfrog: bool = False) -> float:
    """Algorithmic bytes of one forward + adjoint on an n^3 mesh: every 3-D FFT
    one 4-byte read and one write per voxel, every other kernel its distinct
    field inputs and outputs; (382 + 168 W) bytes per voxel, plus 20 per voxel
    for the leapfrog update."""
    return float(n) ** 3 * (382 + 168 * n_webs + (20 if leapfrog else 0))
