"""Shared test helpers: oracle models and mock data for the named workloads."""
import functools

import numpy as np

import fzw_inputs as fi
from oracle.mock import make_counts
from oracle.model import Model, Settings


def workload_at(name, n=None, **cosmo_kw):
    w = fi.workload(name)
    if n is not None and n != w.chains[0].n:
        w = fi.small_variant(w, n)
    if cosmo_kw:
        import dataclasses
        w = dataclasses.replace(w, cosmo=dataclasses.replace(w.cosmo, **cosmo_kw))
    return w


def oracle_model(w, chain=0):
    return Model(Settings.from_workload(w.cosmo, w.web, w.chains[chain]))


@functools.lru_cache(maxsize=16)
def mock_case(name, n=None, tau_sc=None, chain=0, rsd_axis=None):
    """(workload, oracle model, truth nu, eval nu, counts) for a workload."""
    kw = {"tau_sc": tau_sc} if tau_sc is not None else {}
    if rsd_axis is not None:
        kw["rsd_axis"] = rsd_axis
    w = workload_at(name, n, **kw)
    ch = w.chains[chain]
    m = oracle_model(w, chain)
    nu_t = fi.white_noise(ch, fi.ROLE_TRUTH_NU)
    rng = fi.rng_for(ch, fi.ROLE_DATA)
    counts, _ = make_counts(m, nu_t, ch.bias, ch.mean_count,
                            lambda nb, b: fi.gamma_poisson_counts(nb, b, rng))
    nu_e = fi.white_noise(ch, fi.ROLE_EVAL_NU)
    return w, m, nu_t, nu_e, counts


def relnorm(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm((x - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


def bias_entry_error(g, ref):
    """max |g - ref| / max(|ref|, 1e-3 max|ref|) over the table entries."""
    g = np.asarray(g, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    return float(np.max(np.abs(g - ref) / den))


# ------------------------------------------------------------ the parity rule
# Every GPU-vs-oracle comparison follows one rule.
#  * Both sides get the same inputs: the float32 values the GPU is handed
#    (fp32), as float64 for the oracle.
#  * Fixed tolerances: fields 1e-5 normwise, log-likelihood 1e-4 relative,
#    gradients and cotangents 1e-4 normwise, each bias-table entry 1e-4
#    relative to max(|g|, 1e-3 max|g|).
#  * Where the result is ill-conditioned at the state, the tolerance is
#    FLOOR_FACTOR times its conditioning floor instead, the change a float32
#    evaluation may cause that the oracle itself shows:
#      - its movement under a relative perturbation of the input nu of
#        FLOOR_REL (the size of the float32 errors the GPU's fields carry,
#        2-9e-7; the largest over up to FLOOR_DRAWS seeded draws, drawn only
#        while the comparison does not yet pass): normwise for d logL / d nu;
#        for the bias entries the largest movement of any entry, since which
#        entries a rounding moves depends on which particle or cell it carries
#        across a cell face or the density floor, and that particle differs
#        between the draws and the GPU;
#      - for a bias entry, a sum over every voxel, also u32 sum_i |t_i| with
#        t_i the entry's per-voxel terms and u32 = 2^-24 the float32 unit
#        roundoff: the rounding of the terms alone moves the sum by up to
#        that, which is far above 1e-4 |g| where the terms cancel.
FIELD_TOL = 1e-5
LOGL_TOL = 1e-4
GRAD_TOL = 1e-4
FLOOR_REL = 5e-7
FLOOR_DRAWS = 3
FLOOR_FACTOR = 10.0
U32 = 2.0 ** -24


def fp32(a):
    """The float32 rounding of an array, as float64 (what both sides get)."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def oracle_gradient(m, nu, bias, counts):
    """(logL, d/dnu, d/dbias, forward state) of the oracle; the state holds
    the cotangents and the per-entry magnitude sums of the bias gradient."""
    st = m.forward(nu, bias, counts)
    dnu, db = m.adjoint(st)
    return st["logl"], dnu, db, st


class Floor:
    """The oracle's conditioning floor at one state (the rule above); the
    perturbation draws are made lazily."""

    def __init__(self, m, nu, bias, counts, ref_dnu, ref_db, db_abs=None):
        self.args = (m, nu, bias, counts, ref_dnu, ref_db)
        self.rng = np.random.default_rng(99)
        self.nu_f = 0.0
        self.bias_move = np.zeros_like(np.asarray(ref_db, dtype=np.float64))
        self.bias_sum = U32 * np.asarray(db_abs) if db_abs is not None else np.zeros_like(self.bias_move)
        self.draws = 0

    def draw(self):
        m, nu, bias, counts, ref_dnu, ref_db = self.args
        x = nu * (1 + FLOOR_REL * self.rng.standard_normal(nu.shape))
        _, g, b = m.value_and_grad(x, bias, counts)
        self.nu_f = max(self.nu_f, relnorm(g, ref_dnu))
        self.bias_move = np.maximum(self.bias_move, np.abs(b - ref_db).max())
        self.draws += 1

    @property
    def bias_f(self):
        """The largest per-entry floor relative to the entry's scale."""
        ref = np.abs(np.asarray(self.args[5], dtype=np.float64))
        den = np.maximum(ref, 1e-3 * ref.max())
        return float(np.max(np.maximum(self.bias_move, self.bias_sum) / den))

    def _bias_ok(self, g):
        ref = np.asarray(self.args[5], dtype=np.float64)
        den = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
        tol = np.maximum(GRAD_TOL * den, FLOOR_FACTOR * np.maximum(self.bias_move, self.bias_sum))
        return bool(np.all(np.abs(np.asarray(g, dtype=np.float64) - ref) < tol))

    def holds_nu(self, err):
        """d logL / d nu: err (normwise) within GRAD_TOL or FLOOR_FACTOR times
        the floor."""
        while not (err < GRAD_TOL or err < FLOOR_FACTOR * self.nu_f) and self.draws < FLOOR_DRAWS:
            self.draw()
        return err < GRAD_TOL or err < FLOOR_FACTOR * self.nu_f

    def holds_bias(self, g):
        """Every bias entry of g within its tolerance."""
        while not self._bias_ok(g) and self.draws < FLOOR_DRAWS:
            self.draw()
        return self._bias_ok(g)


def conditioned_counts(m, nu, bias, counts, x_min=0.05):
    """The mock counts with every tracer removed from the cells whose density
    (oracle, at state nu) is below x_min times the mean.  There the gradient
    terms scale as 1/x^2, and a cell whose density crosses the floor x_floor
    under float32 rounding changes its term by its full size: at such states
    a float32 path cannot match the float64 gradient, whatever its kernels do.
    Without those tracers every per-voxel term is bounded."""
    x = m.forward(nu, bias)["x"]
    c = np.asarray(counts).copy().reshape(-1)
    c[x < x_min] = 0
    return c.reshape(np.shape(counts))


def off_face(pos, margin=1e-5):
    """Particles whose (redshift-space) position lies more than `margin` cells
    from every cell face: the cloud-in-cell derivative jumps at a face, so a
    particle within float32 noise of one may take the other side's value."""
    f = pos - np.floor(pos)
    return np.minimum(f, 1.0 - f).min(axis=0).ravel() > margin
