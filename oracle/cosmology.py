"""Linear power spectrum and the white-noise filter (oracle, FP64).

Test infrastructure only (see oracle/__init__.py).

The paper states that the white noise is turned into the linear density with
the linear matter power spectrum (Section 2.1, Appendix A) but does not name the
spectrum.  The workloads fix the BBKS transfer function (Bardeen, Bond, Kaiser &
Szalay 1986) with shape parameter Gamma = Omega_m h, primordial tilt n_s and an
amplitude set by sigma8, at z=0 with D=1.

BBKS coefficients are pinned only through their limits (T -> 1 as q -> 0, the
log(q)/q^2 tail); the coefficients themselves are "parity unpinned".
"""
from __future__ import annotations

import numpy as np
from scipy import integrate


def bbks_transfer(k, omega_m: float, h: float):
    """BBKS transfer function, k in h/Mpc."""
    k = np.asarray(k, dtype=np.float64)
    q = k / (omega_m * h)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = (np.log1p(2.34 * q) / (2.34 * q)
             * (1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4) ** -0.25)
    return np.where(q > 0, t, 1.0)


def tophat_window(x):
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        w = 3.0 * (np.sin(x) - x * np.cos(x)) / x ** 3
    return np.where(np.abs(x) > 1e-4, w, 1.0 - x * x / 10.0)


def unnormalised_power(k, cosmo):
    k = np.asarray(k, dtype=np.float64)
    return k ** cosmo.n_s * bbks_transfer(k, cosmo.omega_m, cosmo.h) ** 2


def sigma_r_squared(radius: float, cosmo, amplitude: float = 1.0) -> float:
    """sigma^2(R) = (1/2 pi^2) int dk k^2 P(k) W_TH(kR)^2, by adaptive quadrature
    in ln k over [1e-5, 1e2] h/Mpc."""
    def integrand(lnk):
        k = np.exp(lnk)
        return k ** 3 * amplitude * unnormalised_power(k, cosmo) * tophat_window(k * radius) ** 2

    val, _ = integrate.quad(integrand, np.log(1e-5), np.log(1e2), limit=500,
                            epsabs=0.0, epsrel=1e-11)
    return val / (2.0 * np.pi ** 2)


def power_amplitude(cosmo) -> float:
    """Amplitude A with P(k) = A k^n_s T(k)^2 normalised to sigma8 at 8 Mpc/h."""
    return cosmo.sigma8 ** 2 / sigma_r_squared(8.0, cosmo, 1.0)


def linear_power(k, cosmo, amplitude: float | None = None):
    a = power_amplitude(cosmo) if amplitude is None else amplitude
    return a * unnormalised_power(k, cosmo)


def white_noise_filter(kmag, dx: float, cosmo, amplitude: float | None = None):
    """h(k) = sqrt(P(k) / dx^3) with h(0) = 0 (Appendix A).

    Reading: the printed prefactor of the white-noise map would give a
    covariance scaled by dx^-6, at odds with the covariance the same appendix
    states (dx^-3 F^-1 P F); the prefactor dx^-3/2 is the one consistent with
    that covariance, so delta_L = irfftn(h * rfftn(nu)) with this h.
    """
    kmag = np.asarray(kmag, dtype=np.float64)
    p = linear_power(np.where(kmag > 0, kmag, 1.0), cosmo, amplitude)
    return np.where(kmag > 0, np.sqrt(p / dx ** 3), 0.0)
