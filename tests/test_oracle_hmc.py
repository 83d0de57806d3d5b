"""Leapfrog and Hamiltonian of the oracle (Sections 2.1-2.2)."""
import numpy as np
import pytest

import fzw_inputs as fi
from oracle import hmc
from tests.helpers import mock_case

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def test_leapfrog_harmonic_oscillator_closed_form():
    """For U = q^2/2 and unit mass one kick-drift-kick step is the linear map
    [[1 - e^2/2, e], [-e (1 - e^2/4), 1 - e^2/2]] (Hairer, Lubich & Wanner,
    Geometric Numerical Integration, Sec. I.1); n steps are its n-th power."""
    eps, n = 0.1, 37
    q0, p0 = np.array([0.3, -1.2]), np.array([0.8, 0.1])
    step = np.array([[1 - eps ** 2 / 2, eps], [-eps * (1 - eps ** 2 / 4), 1 - eps ** 2 / 2]])
    mat = np.linalg.matrix_power(step, n)
    gfn = lambda q, u: (0.5 * float(q @ q), q.copy(), np.zeros_like(u))
    q, u, p, pu, h0, h1 = hmc.leapfrog(gfn, q0, np.zeros(1), p0, np.zeros(1), 1.0, 1.0, eps, n)
    want = mat @ np.stack([q0, p0])
    assert np.allclose(q, want[0], atol=1e-14)
    assert np.allclose(p, want[1], atol=1e-14)
    # energy error of leapfrog on the oscillator is O(eps^2)
    assert abs(h1 - h0) < eps ** 2 * h0


def _potential(name="c0fd"):
    w, m, nu_t, nu_e, counts = mock_case(name)
    ch = w.chains[0]
    tying = w.free
    mu = np.full(len(tying), fi.PRIOR_MU_ALPHA)
    sig = np.full(len(tying), fi.PRIOR_SIGMA_ALPHA)
    u0 = np.log(np.array([ch.bias[r[0], c] for r, c in tying]))
    gfn = lambda q, u: hmc.potential_and_grad(m, q, u, ch.bias, tying, mu, sig, counts)
    return gfn, nu_t, u0


def test_leapfrog_reversible_on_the_model():
    gfn, nu, u = _potential()
    rng = np.random.default_rng(4)
    p = rng.standard_normal(nu.shape)
    pu = rng.standard_normal(u.shape)
    minv_u = np.full(u.shape, 1e-3)
    q1, u1, p1, pu1, h0, h1 = hmc.leapfrog(gfn, nu, u, p, pu, 1.0, minv_u, 2e-3, 6)
    q2, u2, p2, pu2, _, _ = hmc.leapfrog(gfn, q1, u1, -p1, -pu1, 1.0, minv_u, 2e-3, 6)
    assert np.allclose(q2, nu, atol=1e-10)
    assert np.allclose(u2, u, atol=1e-12)
    assert np.allclose(-p2, p, atol=1e-8)


def test_leapfrog_energy_error_second_order_smooth_potential():
    """On a smooth anharmonic potential, halving the step at a fixed trajectory
    length divides |dH| by about 4.  (The model's own potential is only
    piecewise smooth: CIC weights have kinks at cell faces and the spherical
    collapse a hinge, so its energy error also carries jumps at crossings.)"""
    rng = np.random.default_rng(5)
    q0 = rng.standard_normal(50)
    p0 = rng.standard_normal(50)
    gfn = lambda q, u: (float(np.sum(q ** 4 / 4 + q ** 2 / 2)), q ** 3 + q, np.zeros_like(u))
    errs = []
    for eps, n in ((0.04, 25), (0.02, 50), (0.01, 100)):
        *_, h0, h1 = hmc.leapfrog(gfn, q0, np.zeros(1), p0, np.zeros(1), 1.0, 0.0, eps, n)
        errs.append(abs(h1 - h0))
    assert 3.0 < errs[0] / errs[1] < 5.0
    assert 3.0 < errs[1] / errs[2] < 5.0


def test_potential_gradient_includes_priors():
    """dU/dnu = -dlogL/dnu + nu and dU/du adds (u - mu)/sigma^2 (central differences)."""
    gfn, nu, u = _potential()
    pot, gnu, gu = gfn(nu, u)
    for i in range(len(u)):
        e = np.zeros_like(u)
        e[i] = 1e-6
        fd = (gfn(nu, u + e)[0] - gfn(nu, u - e)[0]) / 2e-6
        assert fd == pytest.approx(gu[i], rel=1e-5, abs=1e-6 * np.abs(gu).max())


@pytest.mark.parametrize("scheme,order", [("leapfrog", 2), ("blanes2", 2), ("yoshida4", 4)])
def test_integrator_energy_error_order(scheme, order):
    """On a smooth anharmonic potential, halving the step at a fixed
    trajectory length divides |dH| by about 2^order; every scheme's
    coefficients sum to one full kick and one full drift per step."""
    kicks, drifts = hmc.SCHEMES[scheme]
    assert sum(kicks) == pytest.approx(1.0, abs=1e-14) and sum(drifts) == pytest.approx(1.0, abs=1e-14)
    rng = np.random.default_rng(5)
    q0 = rng.standard_normal(50)
    p0 = rng.standard_normal(50)
    gfn = lambda q, u: (float(np.sum(q ** 4 / 4 + q ** 2 / 2)), q ** 3 + q, np.zeros_like(u))
    errs = []
    for eps, n in ((0.04, 25), (0.02, 50), (0.01, 100)):
        *_, h0, h1 = hmc.integrate(gfn, q0, np.zeros(1), p0, np.zeros(1), 1.0, 0.0, eps, n, scheme)
        errs.append(abs(h1 - h0))
    r = 2.0 ** order
    assert 0.7 * r < errs[0] / errs[1] < 1.3 * r
    assert 0.7 * r < errs[1] / errs[2] < 1.3 * r


def test_integrators_are_reversible_and_leapfrog_matches():
    """Each scheme is symmetric: integrating back with negated momenta returns
    to the start; the leapfrog scheme is the kick-drift-kick step."""
    gfn, nu, u = _potential()
    rng = np.random.default_rng(4)
    p = rng.standard_normal(nu.shape)
    pu = rng.standard_normal(u.shape)
    minv_u = np.full(u.shape, 1e-3)
    for scheme in hmc.SCHEMES:
        q1, u1, p1, pu1, h0, h1 = hmc.integrate(gfn, nu, u, p, pu, 1.0, minv_u, 2e-3, 3, scheme)
        q2, u2, p2, pu2, _, _ = hmc.integrate(gfn, q1, u1, -p1, -pu1, 1.0, minv_u, 2e-3, 3, scheme)
        assert np.allclose(q2, nu, atol=1e-10) and np.allclose(u2, u, atol=1e-12)
        assert np.allclose(-p2, p, atol=1e-8)
    a = hmc.integrate(gfn, nu, u, p, pu, 1.0, minv_u, 2e-3, 4, "leapfrog")
    b = hmc.leapfrog(gfn, nu, u, p, pu, 1.0, minv_u, 2e-3, 4)
    for x, y in zip(a, b):
        assert np.allclose(x, y, rtol=1e-13, atol=1e-13)


def test_blanes_scheme_beats_leapfrog_on_a_gaussian_at_equal_cost():
    """The two-stage scheme with b = 0.21178 at step 2 eps has a smaller
    energy error on a Gaussian target than leapfrog at step eps (same number
    of gradients), the property it was designed for."""
    rng = np.random.default_rng(9)
    scales = np.exp(rng.uniform(-1, 0, 200))
    q0 = rng.standard_normal(200) * scales
    p0 = rng.standard_normal(200)
    gfn = lambda q, u: (float(np.sum(0.5 * q * q / scales ** 2)), q / scales ** 2, np.zeros_like(u))
    eps = 0.12
    e_lf, e_b2 = [], []
    for rep in range(20):
        p = np.random.default_rng(rep).standard_normal(200)
        *_, h0, h1 = hmc.integrate(gfn, q0, np.zeros(1), p, np.zeros(1), 1.0, 0.0, eps, 40, "leapfrog")
        e_lf.append(abs(h1 - h0))
        *_, h0, h1 = hmc.integrate(gfn, q0, np.zeros(1), p, np.zeros(1), 1.0, 0.0, 2 * eps, 20, "blanes2")
        e_b2.append(abs(h1 - h0))
    assert np.mean(e_b2) < 0.5 * np.mean(e_lf)


def test_potential_gradient_with_the_full_signed_table():
    """All 64 entries of the 16-region table free, the negative cut-off
    exponents sampled as -exp(u): dU/du by central differences."""
    import dataclasses
    w, m, nu_t, nu_e, counts = mock_case("c2", 16)
    ch = w.chains[0]
    wf = dataclasses.replace(w, free=fi.full_table_free(w.n_regions))
    mu, sig = fi.prior_arrays(wf)
    u = fi.free_start(wf, ch)
    signs = fi.free_signs(wf, ch)
    assert np.any(signs < 0) and len(u) == 64
    assert np.allclose(hmc.tied_table(ch.bias, u, wf.free, signs), ch.bias)
    gfn = lambda q, uu: hmc.potential_and_grad(m, q, uu, ch.bias, wf.free, mu, sig, counts, signs)
    pot, gnu, gu = gfn(nu_t, u)
    rng = np.random.default_rng(3)
    for i in rng.choice(64, size=10, replace=False):
        e = np.zeros_like(u)
        e[i] = 1e-6
        fd = (gfn(nu_t, u + e)[0] - gfn(nu_t, u - e)[0]) / 2e-6
        assert fd == pytest.approx(gu[i], rel=1e-5, abs=1e-6 * np.abs(gu).max())
