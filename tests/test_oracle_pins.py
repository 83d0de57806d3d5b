"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage or closed form it checks.  None of them re-types
the oracle's own formula: they use worked limits, analytic fields, printed
table values, library distributions or brute force.
"""
import json
import os

import numpy as np
import pytest
from scipy import integrate, stats

import fzw_inputs as fi
from oracle import cosmology
from oracle.model import Grid, Model, Settings, nb_loglike, PAIRS
from oracle.stats import power_spectrum

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _model(n=16, box=125.0, **kw):
    kw.setdefault("tau_sc", 0.0)   # the exact spherical-collapse hinge
    cos = fi.Cosmo(**{k: v for k, v in kw.items() if k in fi.Cosmo.__dataclass_fields__})
    web = fi.Web(**{k: v for k, v in kw.items() if k in fi.Web.__dataclass_fields__})
    ch = fi.Chain(n, box, fi.four_class_table(), 1.0, (9, n))
    return Model(Settings.from_workload(cos, web, ch))


def _coords(n, box):
    x = np.arange(n) * box / n
    return np.meshgrid(x, x, x, indexing="ij")


# ------------------------------------------------------------ printed values
def test_table_cases_nyquist_frequencies():
    """Table 'cases': k_nyq = pi/dL and the non-isotropic sqrt(3) k_nyq, as
    printed to two decimals, equal the largest |k_x| and |k| of the oracle's
    wave-vector grid on a 128^3 mesh."""
    gold = json.load(open(os.path.join(GOLD, "table_cases.json")))
    for name in ("TEST1", "TEST2", "TEST3"):
        t = gold[name]
        assert t["L"] / gold["N"] == pytest.approx(t["dL"])
        g = Grid(gold["N"], t["L"])
        kmax = float(np.abs(g.k[0]).max())
        assert round(kmax, 2) == pytest.approx(t["k_nyq"], abs=1e-9)
        assert round(float(g.kmag.max()), 2) == pytest.approx(t["k_nyq_noniso"], abs=0.011)


def test_bias_tables_match_printed_values():
    """Tables 'values' and 'values3' as printed feed the workloads."""
    v = json.load(open(os.path.join(GOLD, "table_values.json")))
    assert tuple(v["TEST1"]["alpha"]) == fi.TEST1_ALPHA
    assert tuple(v["TEST1"]["beta"]) == fi.TEST1_BETA
    assert tuple(v["TEST2"]["alpha"]) == fi.TEST2_ALPHA
    v3 = json.load(open(os.path.join(GOLD, "table_values3.json")))
    assert [tuple(r) for r in v3["rows"]] == [tuple(r) for r in fi.TEST3_TABLE]
    t = fi.sixteen_region_table()
    assert np.allclose(t[:, fi.COL_EPS], -np.array(v3["rows"])[:, 2])
    assert np.allclose(t[:, fi.COL_RHO], np.array(v3["rows"])[:, 3])


# ------------------------------------------------------------ power spectrum
def test_bbks_small_scale_limit():
    """The transfer function tends to 1 on large scales."""
    assert cosmology.bbks_transfer(1e-7, 0.31, 0.68) == pytest.approx(1.0, abs=1e-5)


def _sphere_window(k, radius, nodes=256):
    """Fourier transform of the unit-volume sphere of the given radius,
    computed here by quadrature of its definition: W(k) = (3/R^3) int_0^R r^2
    sin(kr)/(kr) dr (the angular integral of exp(i k.x) over a shell is
    4 pi r^2 sin(kr)/(kr)), Gauss-Legendre in r."""
    x, w = np.polynomial.legendre.leggauss(nodes)
    r = 0.5 * radius * (x + 1.0)
    kr = np.outer(k, r)
    j0 = np.sinc(kr / np.pi)
    return 3.0 / radius ** 3 * (j0 * r * r) @ (0.5 * radius * w)


def test_sigma8_normalisation_independent_window():
    """The amplitude reproduces sigma8 = 0.81: the variance of the linear
    density in spheres of 8 Mpc/h, sigma^2 = (1/2 pi^2) int dk k^2 P(k) W(k)^2,
    with the sphere's window taken from its definition by quadrature (not the
    oracle's closed form) and Simpson's rule in ln k (not the oracle's
    adaptive integrator).  Only the amplitude and the BBKS shape come from the
    oracle; a wrong window or normalisation integral moves sigma8."""
    cos = fi.Cosmo()
    amp = cosmology.power_amplitude(cos)
    lnk = np.linspace(np.log(1e-5), np.log(20.0), 20001)
    k = np.exp(lnk)
    pk = amp * k ** cos.n_s * cosmology.bbks_transfer(k, cos.omega_m, cos.h) ** 2
    win = _sphere_window(k, 8.0)
    assert _sphere_window(np.array([1e-6]), 8.0)[0] == pytest.approx(1.0, abs=1e-9)
    s2 = integrate.simpson(k ** 3 * pk * win ** 2, x=lnk) / (2 * np.pi ** 2)
    assert np.sqrt(s2) == pytest.approx(0.81, rel=1e-4)


def test_white_noise_filter_recovers_input_power():
    """Appendix A: the linear density has covariance dx^-3 F^-1 P F, so the
    binned estimate (dx^3/N^3)|rfftn delta_L|^2 averages to P(k)."""
    m = _model(n=32, box=250.0)
    edges = np.linspace(0.03, 0.35, 9)
    ratios = []
    for seed in range(24):
        nu = np.random.default_rng(seed).standard_normal((32, 32, 32))
        dl = m.g.irfft(m.linear_density_hat(nu))
        k, pk, cnt = power_spectrum(dl, 250.0, edges)
        ratios.append(pk / cosmology.linear_power(k, m.s, m.amp))
    r = np.array(ratios)
    mean = r.mean(0)
    err = r.std(0) / np.sqrt(r.shape[0])
    # bins are narrow enough that P varies little across each one
    assert np.all(np.abs(mean - 1.0) < 4 * err + 0.03), (mean, err)
    assert abs(np.average(mean, weights=1 / err ** 2) - 1.0) < 0.02


def test_white_noise_filter_single_mode_is_eigenfunction():
    """A single Fourier mode is an eigenfunction of the filter with eigenvalue
    h(k) = sqrt(P(k)/dx^3)."""
    n, box = 16, 125.0
    m = _model(n, box)
    x, y, z = _coords(n, box)
    kv = 2 * np.pi / box * np.array([1, 2, 3])
    nu = np.cos(kv[0] * x + kv[1] * y + kv[2] * z)
    dl = m.g.irfft(m.linear_density_hat(nu))
    kk = np.linalg.norm(kv)
    h = np.sqrt(cosmology.linear_power(kk, m.s, m.amp) / (box / n) ** 3)
    assert np.allclose(dl, h * nu, atol=1e-12 * h)


# --------------------------------------------------------------------- ALPT
def _inject(m, dl):
    return m.g.rfft(dl)


def test_zeldovich_plane_wave():
    """Pure 2LPT (r_s -> 0 makes K = 1): delta_L = A cos(k x) has S2 = 0 and the
    Zel'dovich displacement Psi_x = -(A/k) sin(k x), Psi_y = Psi_z = 0."""
    n, box, a = 16, 125.0, 0.7
    m = _model(n, box, r_s=0.0)
    x, y, z = _coords(n, box)
    k = 2 * np.pi / box * 2
    psi, lpt = m.alpt(_inject(m, a * np.cos(k * x)))
    assert np.allclose(lpt["s2"], 0.0, atol=1e-13)
    assert np.allclose(psi[0], -(a / k) * np.sin(k * x), atol=1e-11)
    assert np.allclose(psi[1:], 0.0, atol=1e-11)


def test_2lpt_crossed_waves():
    """Pure 2LPT: delta_L = A cos(kx) + B cos(ky) gives S2 = A B cos kx cos ky and
    Psi_x = -(A/k) sin kx - (3/14)(A B / k) sin kx cos ky (second order with
    D2 = -3/7, from lap phi2 = S2, Psi2 = D2 grad phi2)."""
    n, box, a, b = 16, 125.0, 0.6, 0.4
    m = _model(n, box, r_s=0.0)
    x, y, z = _coords(n, box)
    k = 2 * np.pi / box * 2
    psi, lpt = m.alpt(_inject(m, a * np.cos(k * x) + b * np.cos(k * y)))
    assert np.allclose(lpt["s2"], a * b * np.cos(k * x) * np.cos(k * y), atol=1e-12)
    want = -(a / k) * np.sin(k * x) - (3.0 / 14.0) * (a * b / k) * np.sin(k * x) * np.cos(k * y)
    assert np.allclose(psi[0], want, atol=1e-11)
    want_y = -(b / k) * np.sin(k * y) - (3.0 / 14.0) * (a * b / k) * np.sin(k * y) * np.cos(k * x)
    assert np.allclose(psi[1], want_y, atol=1e-11)


def test_alpt_blend_at_finite_radius_mode_by_mode():
    """Section 2.3 boxed equation: at a finite smoothing radius the ALPT
    displacement is, mode by mode, K(k) times the pure 2LPT displacement plus
    (1 - K(k)) times the pure spherical-collapse one, with the Gaussian
    K = exp(-k^2 r_s^2 / 2) (r_s read as the Gaussian sigma).  The two pure
    displacements come from the same model at r_s = 0 and r_s -> infinity
    (pinned above by the Zel'dovich, crossed-wave and spherical-collapse
    tests); K is computed here from the wave numbers.  A kernel of another
    width, exp(-k^2 r_s^2), is shown to fail by a wide margin."""
    n, box, rs = 32, 128.0, 4.0
    m = _model(n, box, r_s=rs)
    m0 = _model(n, box, r_s=0.0)
    minf = _model(n, box, r_s=1e9)
    nu = np.random.default_rng(21).standard_normal((n, n, n))
    dl_hat = m.linear_density_hat(nu)
    assert np.std(m.g.irfft(dl_hat)) > 1.0          # large enough that SC and 2LPT differ
    psi = m.alpt(dl_hat)[0]
    psi0 = m0.alpt(dl_hat)[0]
    psiinf = minf.alpt(dl_hat)[0]
    kf = 2 * np.pi / box
    f = np.fft.fftfreq(n, 1.0 / n) * kf
    fz = np.fft.rfftfreq(n, 1.0 / n) * kf
    k2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + fz[None, None, :] ** 2
    for width, ok in ((0.5, True), (1.0, False)):
        kern = np.exp(-width * k2 * rs * rs)
        worst = 0.0
        for j in range(3):
            got = np.fft.rfftn(psi[j])
            want = kern * np.fft.rfftn(psi0[j]) + (1.0 - kern) * np.fft.rfftn(psiinf[j])
            worst = max(worst, np.abs(got - want).max() / np.abs(want).max())
        if ok:
            assert worst < 1e-12
        else:
            assert worst > 1e-2
    assert np.abs(psi0 - psiinf).max() > 0.1 * np.abs(psi0).max()


def test_spherical_collapse_one_dimensional_wave():
    """Pure spherical collapse (r_s -> infinity makes K = 0 for k != 0): for
    delta_L = A cos(k x) the displacement is the zero-mean antiderivative of
    3 (sqrt(1 - 2 delta_L / 3) - 1).  The reference integrates that closed-form
    function with a fine 1-D spectral antiderivative."""
    n, box, a = 32, 250.0, 1.0
    m = _model(n, box, r_s=1e9)
    x, y, z = _coords(n, box)
    k = 2 * np.pi / box
    psi, _ = m.alpt(_inject(m, a * np.cos(k * x)))
    fine = 4096
    xf = np.arange(fine) * box / fine
    d = 3 * (np.sqrt(1 - 2 * a * np.cos(k * xf) / 3) - 1)
    dh = np.fft.rfft(d)
    kk = 2 * np.pi / box * np.arange(dh.size)
    anti = np.zeros_like(dh)
    anti[1:] = dh[1:] / (1j * kk[1:])
    ref = np.fft.irfft(anti, n=fine)[:: fine // n]
    assert np.allclose(psi[0][:, 0, 0], ref, atol=1e-6)
    assert np.allclose(psi[1:], 0.0, atol=1e-10)


def test_spherical_collapse_small_amplitude_matches_zeldovich():
    """For small delta_L the spherical-collapse divergence -> -delta_L, so the
    displacement matches the Zel'dovich one to second order in A."""
    n, box, a = 16, 125.0, 1e-4
    m = _model(n, box, r_s=1e9)
    x, y, z = _coords(n, box)
    k = 2 * np.pi / box * 3
    psi, _ = m.alpt(_inject(m, a * np.cos(k * y)))
    assert np.allclose(psi[1], -(a / k) * np.sin(k * y), atol=5e-3 * a / k)


def test_alpt_displacement_curl_free_for_sc():
    """The spherical-collapse displacement is a gradient: d_i Psi_j = d_j Psi_i
    (checked with an 8th-order finite-difference stencil on a smooth field)."""
    n, box = 32, 250.0
    m = _model(n, box, r_s=1e9)
    x, y, z = _coords(n, box)
    k = 2 * np.pi / box
    dl = 0.5 * np.cos(k * x + 0.3) * np.cos(k * y) + 0.3 * np.sin(k * (y + z))
    psi, _ = m.alpt(_inject(m, dl))
    dx = box / n
    c = [4 / 5, -1 / 5, 4 / 105, -1 / 280]

    def d(f, ax):
        return sum(ci * (np.roll(f, -(i + 1), ax) - np.roll(f, i + 1, ax)) for i, ci in enumerate(c)) / dx

    scale = np.abs(psi).max() / dx
    for i in range(3):
        for j in range(i + 1, 3):
            assert np.abs(d(psi[j], i) - d(psi[i], j)).max() < 2e-3 * scale


# ---------------------------------------------------------------------- CIC
def test_cic_unperturbed_lattice_is_uniform():
    m = _model(16)
    rho = m.cic(m.positions(np.zeros((3, 16, 16, 16))))
    assert np.array_equal(rho, np.ones((16, 16, 16)))


def test_cic_constant_shift_is_uniform_and_mass_conserved():
    m = _model(16)
    psi = np.zeros((3, 16, 16, 16))
    psi[0], psi[1], psi[2] = 3.3, -17.9, 0.45 * m.g.dx
    rho = m.cic(m.positions(psi))
    assert np.allclose(rho, 1.0, atol=1e-12)
    rnd = np.random.default_rng(0).normal(scale=20.0, size=(3, 16, 16, 16))
    assert m.cic(m.positions(rnd)).sum() == pytest.approx(16 ** 3, rel=1e-13)


def test_cic_single_particle_weights_and_wrap():
    """Trilinear weights of one particle, including the periodic wrap, by hand."""
    m = _model(8, box=8.0)
    rho = m.cic(np.array([2.25, 3.5, 7.75]).reshape(3, 1, 1, 1))
    want = np.zeros((8, 8, 8))
    for ix, wx in ((2, 0.75), (3, 0.25)):
        for iy, wy in ((3, 0.5), (4, 0.5)):
            for iz, wz in ((7, 0.25), (0, 0.75)):
                want[ix, iy, iz] += wx * wy * wz
    assert np.allclose(rho, want, atol=1e-15)


def test_cic_brute_force_small_mesh():
    """Vectorised CIC equals a plain loop over particles and the 8 nodes."""
    n = 4
    m = _model(n, box=4.0)
    rng = np.random.default_rng(3)
    psi = rng.normal(scale=1.3, size=(3, n, n, n)).clip(-8, 8)
    pos = m.positions(psi)
    want = np.zeros((n, n, n))
    for i in range(n):
        for j in range(n):
            for l in range(n):
                s = pos[:, i, j, l]
                for cx in range(-12, n + 13):
                    for cy in range(-12, n + 13):
                        for cz in range(-12, n + 13):
                            w = 1.0
                            for sc, c in zip(s, (cx, cy, cz)):
                                w *= max(0.0, 1.0 - abs(sc - c))
                            if w > 0:
                                want[cx % n, cy % n, cz % n] += w
    assert np.allclose(m.cic(pos), want, atol=1e-12)


def test_rsd_plane_parallel_displaces_only_the_line_of_sight():
    """Section 2.9 with a plane-parallel line of sight along z and b_v = 1: a
    uniform displacement along z is amplified by (1+f); x and y are untouched."""
    n = 8
    m = _model(n, box=8.0, rsd_axis=2)
    psi = np.zeros((3, n, n, n))
    psi[2] = 0.5
    psi[0] = 0.25
    pos = m.positions(psi)
    grid = np.indices((n, n, n), dtype=float)
    assert np.allclose(pos[2] - grid[2], 0.5 * (1 + m.s.f_growth))
    assert np.allclose(pos[0] - grid[0], 0.25)


def test_rsd_radial_moves_particles_along_the_observer_ray():
    """Section 2.9 with the observer at the box centre and b_v = 1: each
    particle stays on the ray from the observer through its real-space
    position, its distance from the observer grows by the line-of-sight
    component of f Psi, and on the line of sight through the centre along z
    the shift equals the plane-parallel one."""
    n, box = 8, 16.0
    m = _model(n, box=box, rsd_axis=fi.RSD_RADIAL)
    rng = np.random.default_rng(5)
    psi = 0.6 * rng.standard_normal((3, n, n, n))
    grid = np.indices((n, n, n), dtype=float)
    x = grid + psi / m.g.dx - n / 2
    s = m.positions(psi) - n / 2
    xv, sv = x.reshape(3, -1).T, s.reshape(3, -1).T
    assert np.allclose(np.cross(xv, sv), 0.0, atol=1e-12)
    dist = np.linalg.norm(xv, axis=1)
    vlos = np.einsum("pi,pi->p", m.s.f_growth * psi.reshape(3, -1).T / m.g.dx, xv) / dist
    ahead = dist + vlos > 0
    assert ahead.mean() > 0.9
    assert np.allclose(np.linalg.norm(sv, axis=1)[ahead], (dist + vlos)[ahead], atol=1e-12)
    # the line x = y = n/2 with Psi along z only: radial equals plane-parallel
    pz = np.zeros((3, n, n, n))
    pz[2] = psi[2]
    mp = _model(n, box=box, rsd_axis=2)
    c = n // 2
    assert np.allclose(m.positions(pz)[:, c, c, :], mp.positions(pz)[:, c, c, :], atol=1e-12)
    assert not np.allclose(m.positions(pz), mp.positions(pz))
    # CIC keeps the mass
    assert m.cic(m.positions(psi)).mean() == pytest.approx(1.0, abs=1e-13)


# ---------------------------------------------------------------- web tensors
def test_tidal_tensor_of_plane_wave_is_rank_one():
    """Phi-web with no smoothing: delta = A cos(k.x) has T = A cos(k.x) khat khat^T,
    so the sorted eigenvalues are {A cos, 0, 0} up to order."""
    n, box, a = 16, 100.0, 0.8
    m = _model(n, box)
    x, y, z = _coords(n, box)
    kv = 2 * np.pi / box * np.array([1.0, 2.0, 0.0])
    ph = kv[0] * x + kv[1] * y
    t6 = m.web_tensors(m.g.rfft(a * np.cos(ph)))[0]
    kh = kv / np.linalg.norm(kv)
    for (i, j), c in zip(PAIRS, t6):
        assert np.allclose(c, a * np.cos(ph) * kh[i] * kh[j], atol=1e-12)
    lam, _ = m.eigen(t6)
    want = np.sort(np.stack([a * np.cos(ph).ravel(), 0 * ph.ravel(), 0 * ph.ravel()], 1), 1)[:, ::-1]
    assert np.allclose(lam, want, atol=1e-12)


def test_tidal_tensor_axis_separable_field_is_diagonal():
    n, box = 16, 100.0
    m = _model(n, box)
    x, y, z = _coords(n, box)
    k = 2 * np.pi / box * 2
    amps = (0.3, -0.5, 0.9)
    dl = amps[0] * np.cos(k * x) + amps[1] * np.cos(k * y) + amps[2] * np.cos(k * z)
    t6 = m.web_tensors(m.g.rfft(dl))[0]
    for c, v, a in zip(t6[:3], (x, y, z), amps):
        assert np.allclose(c, a * np.cos(k * v), atol=1e-12)
    for c in t6[3:]:
        assert np.allclose(c, 0.0, atol=1e-12)


def test_delta_web_tensor_is_minus_scaled_hessian():
    """delta-web (no smoothing): T_ij = -ell^2 d_i d_j delta; for A cos(kx),
    T_xx = ell^2 k^2 A cos(kx)."""
    n, box, a, ell = 16, 100.0, 0.4, 2.0
    m = _model(n, box, kinds=(fi.WEB_DELTA,), smooth_r=(0.0,), ell=(ell,))
    x, y, z = _coords(n, box)
    k = 2 * np.pi / box * 3
    t6 = m.web_tensors(m.g.rfft(a * np.cos(k * x)))[0]
    assert np.allclose(t6[0], ell ** 2 * k ** 2 * a * np.cos(k * x), atol=1e-12)
    assert np.allclose(np.stack(t6[1:]), 0.0, atol=1e-12)


def test_gaussian_smoothing_of_tensor_single_mode():
    """A Gaussian smoothing of radius R multiplies a single mode by exp(-k^2 R^2/2)."""
    n, box, a, r = 16, 100.0, 0.4, 8.0
    m = _model(n, box, smooth_r=(r,))
    x, y, z = _coords(n, box)
    k = 2 * np.pi / box * 2
    t6 = m.web_tensors(m.g.rfft(a * np.cos(k * z)))[0]
    assert np.allclose(t6[2], np.exp(-0.5 * k * k * r * r) * a * np.cos(k * z), atol=1e-12)


def test_eigenvalues_invariants_and_rotations():
    """Appendix B: sum of eigenvalues = trace (I1), product = determinant (I3),
    and a rotated diagonal matrix gives back its diagonal, sorted descending."""
    rng = np.random.default_rng(5)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    d = np.array([0.7, -0.2, 0.1])
    mat = q @ np.diag(d) @ q.T
    t6 = [np.full((1, 1, 1), mat[i, j]) for (i, j) in PAIRS]
    lam, _ = _model(4, 4.0).eigen(t6)
    assert np.allclose(lam[0], [0.7, 0.1, -0.2], atol=1e-14)
    a = rng.normal(size=(50, 3, 3))
    a = a + a.transpose(0, 2, 1)
    t6 = [a[:, i, j].reshape(50, 1, 1) for (i, j) in PAIRS]
    lam, _ = _model(4, 4.0).eigen(t6)
    assert np.all(np.diff(lam, axis=1) <= 0)
    assert np.allclose(lam.sum(1), np.trace(a, axis1=1, axis2=2))
    assert np.allclose(lam.prod(1), np.linalg.det(a))


# --------------------------------------------------------- fuzzy memberships
def test_memberships_partition_of_unity_and_hard_limit():
    """Eq. 'soft_cweb_p' memberships are non-negative and sum to one; with a huge
    steepness they become one-hot on the class W = number of eigenvalues above
    the threshold (Eq. 'hard_cweb'), W = 0..3 -> void, sheet, filament, knot."""
    rng = np.random.default_rng(7)
    lam = np.sort(rng.normal(scale=0.5, size=(5000, 3)), 1)[:, ::-1]
    m = _model(4, 4.0)
    _, p = m.memberships(lam)
    assert np.all(p >= -1e-15)
    assert np.allclose(p.sum(0), 1.0)
    hard = _model(4, 4.0, steepness=1e6)
    _, ph = hard.memberships(lam)
    w_class = (lam > hard.s.lambda_th).sum(1)
    ok = np.abs(lam - hard.s.lambda_th).min(1) > 1e-3
    assert ok.sum() > 4000
    onehot = np.eye(4)[w_class]
    assert np.allclose(ph.T[ok], onehot[ok], atol=1e-12)


def _separable_case(n=16, box=100.0, amps=(0.3, -0.25, 0.2), mode=2):
    """delta = sum_j a_j cos(k x_j): every Fourier mode lies on one axis, so
    the web tensors of either kind (no smoothing) are diagonal, with entries
    a_j cos(k x_j) (Phi-web: k_j k_j / k^2 = 1) and ell^2 k^2 a_j cos(k x_j)
    (delta-web)."""
    x, y, z = _coords(n, box)
    k = 2 * np.pi / box * mode
    diag = [a * np.cos(k * v) for a, v in zip(amps, (x, y, z))]
    return k, sum(diag), diag


def _closed_form_f(webs_diag, table, steep, th, x):
    """f at every voxel from the paper's equations, given the diagonal
    entries of each web's tensor: eigenvalues sorted descending (Appendix B
    order), sigmoid weights w_n = 1/(1 + exp(-s (lambda_n - th)))
    (Eq. 'sigmoid'), memberships V, S, F, K = 1-w1, w1-w2, w2-w3, w3
    (Eq. 'soft_cweb_p'), regions p_jk = p_j p_k over two webs, parameters
    interpolated as sum_r p_r theta_r (boxed equation of Section 2.8), then
    f = x^alpha exp(-(x/rho)^eps) (Eq. 'local_bias').  Returns f, the
    region probabilities and the per-region f values."""
    ps = []
    for diag in webs_diag:
        lam = -np.sort(-np.stack([d.ravel() for d in diag], axis=1), axis=1)
        w = 1.0 / (1.0 + np.exp(-steep * (lam - th)))
        ps.append(np.stack([1.0 - w[:, 0], w[:, 0] - w[:, 1], w[:, 1] - w[:, 2], w[:, 2]]))
    preg = ps[0] if len(ps) == 1 else np.einsum("jm,km->jkm", ps[0], ps[1]).reshape(16, -1)
    alpha, eps, rho = [(preg * table[:, c][:, None]).sum(0) for c in (0, 1, 2)]
    f = x ** alpha * np.exp(-(x / rho) ** eps)
    f_r = np.stack([x ** a * np.exp(-(x / r) ** e) for a, e, r in table[:, :3]])
    return f, preg, f_r


def test_parameter_interpolation_soft_memberships():
    """Boxed equation of Section 2.8: the bias parameters (alpha, eps, rho,
    beta) are interpolated per voxel with the region memberships and f is
    evaluated once with them.  On an axis-separable field the eigenvalues are
    known in closed form, so f follows from the paper's equations alone; with
    an unequal table and steepness 20 many voxels sit between classes, and
    mixing the per-region values f_r instead of the parameters misses by far
    more than the tolerance (checked)."""
    n, box = 16, 100.0
    m = _model(n, box)
    k, delta, diag = _separable_case(n, box)
    table = np.array([[0.9, -0.5, 0.10, 2.0], [1.1, -1.0, 0.20, 4.0],
                      [1.4, -2.0, 0.40, 6.0], [1.8, -3.0, 0.60, 8.0]])
    got = m.web_bias(delta, table)
    x = 1.0 + delta.ravel()
    f, preg, f_r = _closed_form_f([diag], table, m.s.steepness, m.s.lambda_th, x)
    assert np.allclose(got["preg"], preg, rtol=0, atol=1e-12)
    assert np.allclose(got["f"], f, rtol=1e-11, atol=0)
    mixed = (preg * f_r).sum(0)
    assert np.abs(mixed / f - 1).max() > 1e-2
    soft = (preg.max(0) < 0.9).mean()
    assert soft > 0.2                                  # a fifth of the voxels are fuzzy


def test_parameter_interpolation_sixteen_regions():
    """The two-web model (Phi-web x delta-web, region 4 j + k): with an
    unequal 16-row table, f at steepness 20 follows the closed form of the
    products of the two webs' memberships, and at steepness 10^6 every voxel
    (eigenvalues off the threshold) takes the f of its hard region, whose web
    classes count the eigenvalues above the threshold (Eq. 'hard_cweb')."""
    n, box, ell = 16, 100.0, 11.25     # ell^2 k^2 = 2: the delta-web classes differ from the Phi-web ones
    # entries a_j cos(k x_j) take the values a_j {+-1, +-0.707, 0}: amplitudes
    # that put Phi-web entries on both sides of the threshold
    k, delta, diag = _separable_case(n, box, amps=(0.12, -0.13, 0.09))
    kw = dict(kinds=(fi.WEB_PHI, fi.WEB_DELTA), smooth_r=(0.0, 0.0), ell=(0.0, ell))
    rng = np.random.default_rng(31)
    table = np.stack([rng.uniform(0.8, 1.8, 16), -rng.uniform(0.5, 3.0, 16), rng.uniform(0.1, 0.6, 16),
                      rng.uniform(2.0, 9.0, 16)], axis=1)
    ddiag = [ell * ell * k * k * d for d in diag]
    x = 1.0 + delta.ravel()
    soft = _model(n, box, **kw)
    f, preg, f_r = _closed_form_f([diag, ddiag], table, soft.s.steepness, soft.s.lambda_th, x)
    assert np.allclose(soft.web_bias(delta, table)["f"], f, rtol=1e-11, atol=0)
    assert np.abs((preg * f_r).sum(0) / f - 1).max() > 1e-2
    hard = _model(n, box, steepness=1e6, **kw)
    th = hard.s.lambda_th
    cls = []
    margin = np.full(n ** 3, np.inf)
    for dg in (diag, ddiag):
        vals = np.stack([d.ravel() for d in dg], axis=1)
        cls.append((vals > th).sum(1))
        margin = np.minimum(margin, np.abs(vals - th).min(1))
    region = 4 * cls[0] + cls[1]
    ok = margin > 1e-4
    assert ok.mean() > 0.9 and len(np.unique(region[ok])) >= 6
    want = f_r[region, np.arange(n ** 3)]
    assert np.allclose(hard.web_bias(delta, table)["f"][ok], want[ok], rtol=1e-12, atol=0)


def test_sixteen_regions_partition_of_unity():
    rng = np.random.default_rng(8)
    m = _model(4, 4.0)
    _, pa = m.memberships(np.sort(rng.normal(size=(100, 3)), 1)[:, ::-1])
    _, pb = m.memberships(np.sort(rng.normal(size=(100, 3)), 1)[:, ::-1])
    p16 = Model.regions([pa, pb])
    assert p16.shape == (16, 100)
    assert np.allclose(p16.sum(0), 1.0)
    assert np.allclose(p16[4 * 2 + 1], pa[2] * pb[1])


# ---------------------------------------------------------------- likelihood
def test_negative_binomial_matches_scipy():
    """Section 2.7: Gamma(beta, nbar/beta) x Poisson is NB(n; r=beta, p=beta/(beta+nbar))."""
    rng = np.random.default_rng(11)
    n = rng.integers(0, 80, size=2000).astype(float)
    nbar = np.exp(rng.normal(0.0, 1.5, size=2000))
    beta = rng.uniform(0.5, 20.0, size=2000)
    ell, _ = nb_loglike(n, np.log(nbar), beta)
    ref = stats.nbinom.logpmf(n, beta, beta / (beta + nbar))
    assert np.allclose(ell, ref, rtol=1e-10, atol=1e-10)


def test_negative_binomial_poisson_limit():
    """beta -> infinity recovers the Poisson likelihood."""
    n = np.arange(0, 30, dtype=float)
    nbar = np.full_like(n, 3.7)
    ell, _ = nb_loglike(n, np.log(nbar), np.full_like(n, 1e9))
    assert np.allclose(ell, stats.poisson.logpmf(n, nbar), atol=1e-6)


def test_gamma_poisson_mock_moments():
    """Mock counts have mean nbar and variance nbar + nbar^2/beta."""
    rng = np.random.default_rng(12)
    nbar = np.full(400_000, 2.0)
    c = fi.gamma_poisson_counts(nbar, np.full_like(nbar, 3.0), rng).astype(float)
    assert c.mean() == pytest.approx(2.0, rel=0.01)
    assert c.var() == pytest.approx(2.0 + 4.0 / 3.0, rel=0.02)


def _counts(m, seed=0, mean=1.0):
    rng = np.random.default_rng(seed)
    return rng.poisson(mean, size=(m.s.n,) * 3).astype(np.uint16)


def test_normalisation_sums_to_number_of_tracers():
    """Eq. 'local_bias': C is fixed by sum nbar = sum n* = N_tr."""
    m = _model(16)
    nu = np.random.default_rng(1).standard_normal((16,) * 3)
    c = _counts(m)
    st = m.forward(nu, fi.four_class_table(), c)
    assert st["nbar"].sum() == pytest.approx(float(c.sum()), rel=1e-12)


def test_equal_regions_make_the_web_irrelevant():
    """With identical parameters in every region the memberships drop out and
    nbar = N_tr f / sum f with f = x^alpha exp(-(x/rho)^eps), x = 1 + delta."""
    m = _model(16)
    nu = np.random.default_rng(2).standard_normal((16,) * 3)
    c = _counts(m)
    tab = fi.four_class_table(alpha=(1.2,) * 4, eps=-1.3, rho=0.3, beta=4.0)
    # no tracers where the model density underflows (scipy's pmf would be -inf)
    c[m.forward(nu, tab)["rho"] < 0.05] = 0
    st = m.forward(nu, tab, c)
    x = np.maximum(st["rho"].ravel(), 1e-6)
    f = x ** 1.2 * np.exp(-(x / 0.3) ** -1.3)
    want = c.sum() * f / f.sum()
    assert np.allclose(st["nbar"], want, rtol=1e-10, atol=1e-300)
    ref = stats.nbinom.logpmf(c.ravel(), 4.0, 4.0 / (4.0 + want))
    assert st["logl"] == pytest.approx(ref.sum(), rel=1e-10)


# ---------------------------------------------------------------- Wiener start
def test_wiener_start_is_the_gaussian_posterior_mean():
    """Section 2.2 initialisation: on a 4^3 mesh, the oracle's Fourier-diagonal
    Wiener filter equals the textbook posterior mean of nu under nu ~ N(0, I),
    delta_tr = L nu + shot noise of variance 1/nbar per cell, written with
    dense matrices: E[nu | d] = L^T (L L^T + I/nbar)^-1 d, where L is the
    linear-density operator built column by column from the model."""
    from oracle import wiener
    n = 4
    m = _model(n, box=40.0)
    rng = np.random.default_rng(8)
    counts = rng.poisson(1.5, size=(n, n, n))
    dim = n ** 3
    cols = []
    for i in range(dim):
        e = np.zeros(dim)
        e[i] = 1.0
        cols.append(m.g.irfft(m.linear_density_hat(e.reshape(n, n, n))).ravel())
    L = np.stack(cols, axis=1)
    nbar = counts.sum() / dim
    d = wiener.tracer_contrast(counts).ravel()
    want = L.T @ np.linalg.solve(L @ L.T + np.eye(dim) / nbar, d)
    got = wiener.wiener_white_noise(m, counts).ravel()
    assert np.allclose(got, want, rtol=1e-9, atol=1e-12 * np.abs(want).max())
    assert abs(wiener.tracer_contrast(counts).mean()) < 1e-14


# ---------------------------------------------------------------- validation statistics
def _unit_modes(n, seed):
    rng = np.random.default_rng(seed)
    s = np.fft.rfftn(rng.standard_normal((n, n, n)))
    s = s / np.abs(s)
    s[0, 0, 0] = 0.0
    return s


def test_multipoles_of_a_kaiser_field_match_the_linear_theory_ratios():
    """A field whose every mode has |delta_k| = 1 + f mu^2 (mu = k_z/k) has,
    in the continuum limit, P0 proportional to 1 + 2f/3 + f^2/5 and P2 to
    4f/3 + 4f^2/7 (Kaiser 1987; Hamilton 1992); shells with thousands of modes
    reach it to a few 1e-3."""
    from oracle import stats
    n, box, f = 48, 300.0, 0.6
    s = _unit_modes(n, 3)
    kf = 2 * np.pi / box
    nf = np.fft.fftfreq(n, 1.0 / n)
    nz = np.fft.rfftfreq(n, 1.0 / n)
    k = np.sqrt(nf[:, None, None] ** 2 + nf[None, :, None] ** 2 + nz[None, None, :] ** 2)
    mu = np.where(k > 0, nz[None, None, :] / np.where(k > 0, k, 1.0), 0.0)
    delta = np.fft.irfftn(s * (1 + f * mu * mu), s=(n, n, n), axes=(0, 1, 2))
    km, cnt, p0, p2 = stats.multipoles(delta, None, box, 8 * kf, 4 * kf, 3)
    unit = (box / n) ** 3 / n ** 3
    assert np.all(cnt > 3000)
    assert np.allclose(p0 / unit, 1 + 2 * f / 3 + f * f / 5, rtol=5e-3)
    assert np.allclose(p2 / unit, 4 * f / 3 + 4 * f * f / 7, rtol=1e-2)
    # an isotropic field has no quadrupole beyond the shell's discreteness
    iso = np.fft.irfftn(s, s=(n, n, n), axes=(0, 1, 2))
    _, _, q0, q2 = stats.multipoles(iso, None, box, 8 * kf, 4 * kf, 3)
    assert np.allclose(q0 / unit, 1.0, rtol=1e-12)
    assert np.all(np.abs(q2 / unit) < 5e-3)


def test_cross_correlation_and_propagator_of_scaled_fields():
    from oracle import stats
    n, box = 16, 100.0
    a = np.random.default_rng(4).standard_normal((n, n, n))
    kf = 2 * np.pi / box
    c, g = stats.cross_statistics(3.0 * a, a, box, kf, kf, 5)
    assert np.allclose(c, 1.0, rtol=1e-12) and np.allclose(g, 3.0, rtol=1e-12)
    c, g = stats.cross_statistics(-a, a, box, kf, kf, 5)
    assert np.allclose(c, -1.0, rtol=1e-12) and np.allclose(g, -1.0, rtol=1e-12)


def test_bispectrum_estimator_equals_the_brute_force_triangle_sum():
    """The FFT estimator against the direct sum over every closed triangle of
    DFT modes (k1 + k2 + k3 = 0 on the periodic grid) with |k_i| in the three
    shells, on a 12^3 mesh: B = dx^6/N^3 * mean(d1 d2 d3), and the count."""
    from oracle import stats
    n, box = 12, 60.0
    rng = np.random.default_rng(6)
    g = rng.standard_normal((n, n, n))
    delta = g + 0.4 * (g * g - 1.0)
    kf = 2 * np.pi / box
    k1, k2, dk = 2.0 * kf, 3.0 * kf, 1.0 * kf
    thetas = np.array([0.4, 1.3, 2.2, 2.9])
    k3s, b, q, tri = stats.bispectrum(delta, box, k1, k2, dk, thetas)
    full = np.fft.fftn(delta)
    idx = np.arange(n)
    fr = np.where(idx <= n // 2, idx, idx - n)
    grid = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), -1).reshape(-1, 3)
    kmag = kf * np.sqrt(np.sum(fr[grid] ** 2, axis=1))

    def shell(kc):
        return grid[(kmag >= kc - 0.5 * dk) & (kmag < kc + 0.5 * dk)]
    s1, s2 = shell(k1), shell(k2)
    dx = box / n
    for k3, bb, tt in zip(k3s, b, tri):
        lo, hi = k3 - 0.5 * dk, k3 + 0.5 * dk
        tot, cnt = 0.0, 0
        for a1 in s1:
            a3 = (-(a1[None, :] + s2)) % n
            m3 = kf * np.sqrt(np.sum(fr[a3] ** 2, axis=1))
            ok = (m3 >= lo) & (m3 < hi)
            if np.any(ok):
                tot += np.sum(full[a1[0], a1[1], a1[2]] * full[s2[ok, 0], s2[ok, 1], s2[ok, 2]]
                              * full[a3[ok, 0], a3[ok, 1], a3[ok, 2]]).real
                cnt += int(np.sum(ok))
        assert cnt > 0
        assert tt == pytest.approx(cnt, rel=1e-9)
        assert bb == pytest.approx(dx ** 6 / n ** 3 * tot / cnt, rel=1e-9)
