"""The oracle's hand-written adjoint against central finite differences (FP64)
and against automatic differentiation of an independent PyTorch forward."""
import numpy as np
import pytest

from tests.helpers import mock_case
from tests.torch_reference import value_and_grad_torch

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

RADIAL = 3   # radial RSD about the box centre
CASES = [("c0fd", None, 0.0, None), ("c2", 16, 0.0, None), ("c0fd", None, 0.05, None),
         ("c2", 16, 0.0, RADIAL)]
# finite-difference steps (truth point, evaluation point) per case, each inside
# the range where the central difference has converged for these seeds
STEPS = {("c0fd", 0.0, None): (1e-7, 1e-6), ("c2", 0.0, None): (1e-7, 1e-7),
         ("c0fd", 0.05, None): (1e-7, 1e-6), ("c2", 0.0, RADIAL): (1e-7, 1e-7)}


def _fd(m, nu, bias, counts, dnu=None, dbias=None, h=1e-7):
    nu_p = nu + h * dnu if dnu is not None else nu
    nu_m = nu - h * dnu if dnu is not None else nu
    b_p = bias + h * dbias if dbias is not None else bias
    b_m = bias - h * dbias if dbias is not None else bias
    return (m.forward(nu_p, b_p, counts)["logl"] - m.forward(nu_m, b_m, counts)["logl"]) / (2 * h)


@pytest.mark.parametrize("name,n,tau,rsd", CASES)
@pytest.mark.parametrize("which", ["truth", "eval"])
def test_gradient_directional_fd(name, n, tau, rsd, which):
    """Central differences with a small step: the spherical-collapse hinge and
    the CIC cell faces make the map only piecewise smooth, so the step is kept
    well below the distance of the nearest kink in these fixed seeds."""
    w, m, nu_t, nu_e, counts = mock_case(name, n, tau, rsd_axis=rsd)
    nu = nu_t if which == "truth" else nu_e
    bias = w.chains[0].bias
    logl, dnu, dbias = m.value_and_grad(nu, bias, counts)
    rng = np.random.default_rng(17)
    # the evaluation point has |logL| ~ 1e5 (tracers in empty cells), so its
    # step is larger to keep the round-off of the difference small
    h = STEPS[(name, tau, rsd)][0 if which == "truth" else 1]
    for _ in range(3):
        v = rng.standard_normal(nu.shape)
        fd = _fd(m, nu, bias, counts, dnu=v, h=h)
        assert fd == pytest.approx(float(np.sum(dnu * v)), rel=1e-5,
                                   abs=1e-7 * np.linalg.norm(dnu) + 50 * 1e-16 * abs(logl) / h)


@pytest.mark.parametrize("name,n,tau,rsd", CASES[:2] + CASES[3:])
def test_gradient_coordinates_fd(name, n, tau, rsd):
    """64 random voxels of d logL / d nu, each by central differences."""
    w, m, nu_t, nu_e, counts = mock_case(name, n, tau, rsd_axis=rsd)
    bias = w.chains[0].bias
    logl, dnu, _ = m.value_and_grad(nu_t, bias, counts)
    rng = np.random.default_rng(23)
    idx = rng.choice(nu_t.size, size=64, replace=False)
    scale = np.abs(dnu).max()
    for i in idx:
        e = np.zeros(nu_t.size)
        e[i] = 1.0
        fd = _fd(m, nu_t, bias, counts, dnu=e.reshape(nu_t.shape))
        assert fd == pytest.approx(dnu.ravel()[i], rel=1e-5, abs=1e-6 * scale + 50e-16 * abs(logl) / 1e-7)


@pytest.mark.parametrize("name,n,tau,rsd", CASES[:2] + CASES[3:])
def test_bias_table_gradient_fd(name, n, tau, rsd):
    w, m, nu_t, nu_e, counts = mock_case(name, n, tau, rsd_axis=rsd)
    bias = w.chains[0].bias
    logl, _, dbias = m.value_and_grad(nu_t, bias, counts)
    scale = np.abs(dbias).max()
    for r in range(bias.shape[0]):
        for c in range(4):
            e = np.zeros_like(bias)
            e[r, c] = 1.0
            fd = _fd(m, nu_t, bias, counts, dbias=e, h=1e-5)
            assert fd == pytest.approx(dbias[r, c], rel=1e-5, abs=1e-7 * scale + 50e-16 * abs(logl) / 1e-5)


@pytest.mark.parametrize("name,n,tau,rsd", CASES)
def test_adjoint_matches_torch_autodiff(name, n, tau, rsd):
    """Element-wise agreement of logL, d/d nu and d/d bias with reverse-mode
    autodiff of an independent float64 PyTorch forward."""
    w, m, nu_t, nu_e, counts = mock_case(name, n, tau, rsd_axis=rsd)
    bias = w.chains[0].bias
    for nu in (nu_t, nu_e):
        logl, dnu, dbias = m.value_and_grad(nu, bias, counts)
        lt, dnu_t, dbias_t = value_and_grad_torch(m, nu, bias, counts)
        assert logl == pytest.approx(lt, rel=1e-11)
        assert np.allclose(dnu, dnu_t, rtol=1e-8, atol=1e-9 * np.abs(dnu_t).max())
        assert np.allclose(dbias, dbias_t, rtol=1e-8, atol=1e-9 * np.abs(dbias_t).max())
