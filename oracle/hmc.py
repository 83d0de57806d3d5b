"""Posterior potential, Hamiltonian and leapfrog (oracle, FP64).

Test infrastructure only (see oracle/__init__.py).

Section 2.1 (Eq. 'posterior', Eq. 'lognormal'): whitened Gaussian prior on nu and
log-normal priors on the free bias parameters.  Sampling u = ln b, the density
of u is Gaussian with mean mu and width sigma (the 1/b of the log-normal
cancels the Jacobian).  Potential (additive constants dropped):
    U = -logL + |nu|^2 / 2 + sum_f (u_f - mu_f)^2 / (2 sigma_f^2)
Section 2.2: HMC with a diagonal mass matrix; kick-drift-kick leapfrog,
H = U + p^T M^-1 p / 2.
"""
from __future__ import annotations

import numpy as np


def tied_table(base, u, tying, signs=None):
    """Bias table with every entry listed for free parameter f set to
    s_f exp(u_f) (s_f = +1 unless `signs` is given: a signed parameter such as
    a negative cut-off exponent is sampled through the log of its magnitude).
    `tying` is a list of (region tuple, column) per free parameter."""
    t = np.array(base, dtype=np.float64, copy=True)
    for fi, (regions, col) in enumerate(tying):
        s = 1.0 if signs is None else float(signs[fi])
        for r in regions:
            t[r, col] = s * np.exp(u[fi])
    return t


def potential_and_grad(model, nu, u, base, tying, mu, sigma, counts, signs=None):
    table = tied_table(base, u, tying, signs)
    logl, dnu, dtab = model.value_and_grad(nu, table, counts)
    uu = np.asarray(u, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    pot = -logl + 0.5 * float(np.sum(nu * nu)) + float(np.sum((uu - mu) ** 2 / (2 * sigma ** 2)))
    gnu = -dnu + nu
    gu = np.zeros_like(uu)
    for fi, (regions, col) in enumerate(tying):
        s = 1.0 if signs is None else float(signs[fi])
        gu[fi] = -sum(dtab[r, col] for r in regions) * s * np.exp(uu[fi])
    gu += (uu - mu) / sigma ** 2
    return pot, gnu, gu


def kinetic(p_nu, p_u, minv_nu, minv_u):
    return 0.5 * float(np.sum(minv_nu * p_nu * p_nu)) + 0.5 * float(np.sum(minv_u * p_u * p_u))


def leapfrog(grad_fn, q_nu, q_u, p_nu, p_u, minv_nu, minv_u, eps, n_steps):
    """Kick-drift-kick leapfrog.  `grad_fn(q_nu, q_u) -> (U, dU/dnu, dU/du)`.
    Returns the end state and (H_start, H_end)."""
    q_nu, q_u = np.array(q_nu, dtype=np.float64), np.array(q_u, dtype=np.float64)
    p_nu, p_u = np.array(p_nu, dtype=np.float64), np.array(p_u, dtype=np.float64)
    pot, g_nu, g_u = grad_fn(q_nu, q_u)
    h0 = pot + kinetic(p_nu, p_u, minv_nu, minv_u)
    for _ in range(n_steps):
        p_nu -= 0.5 * eps * g_nu
        p_u -= 0.5 * eps * g_u
        q_nu += eps * minv_nu * p_nu
        q_u += eps * minv_u * p_u
        pot, g_nu, g_u = grad_fn(q_nu, q_u)
        p_nu -= 0.5 * eps * g_nu
        p_u -= 0.5 * eps * g_u
    h1 = pot + kinetic(p_nu, p_u, minv_nu, minv_u)
    return q_nu, q_u, p_nu, p_u, h0, h1


# Splitting integrators (Section 2.2 names second- and fourth-order HMC and
# the variant of Blanes, Casas & Sanz-Serna 2014).  One step is
#   K(a_0) D(b_1) K(a_1) ... D(b_m) K(a_m)
# with K(a) the kick p -= a eps dU/dq and D(b) the drift q += b eps M^-1 p,
# and the gradient evaluated after every drift.
_W1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
_W0 = -(2.0 ** (1.0 / 3.0)) * _W1
_B2 = 0.21178
SCHEMES = {
    # kick-drift-kick (second order, one gradient per step)
    "leapfrog": ((0.5, 0.5), (1.0,)),
    # two-stage splitting with b = 0.21178, minimising the energy error of
    # Gaussian targets (Blanes, Casas & Sanz-Serna 2014; two gradients)
    "blanes2": ((_B2, 1.0 - 2.0 * _B2, _B2), (0.5, 0.5)),
    # fourth order: three leapfrog steps of w1, w0, w1 (Yoshida 1990;
    # Forest & Ruth 1990), adjacent kicks merged (three gradients)
    "yoshida4": ((0.5 * _W1, 0.5 * (_W1 + _W0), 0.5 * (_W0 + _W1), 0.5 * _W1), (_W1, _W0, _W1)),
}


def integrate(grad_fn, q_nu, q_u, p_nu, p_u, minv_nu, minv_u, eps, n_steps, scheme="leapfrog"):
    """n_steps of a splitting scheme from SCHEMES; same arguments and returns
    as `leapfrog`."""
    kicks, drifts = SCHEMES[scheme]
    q_nu, q_u = np.array(q_nu, dtype=np.float64), np.array(q_u, dtype=np.float64)
    p_nu, p_u = np.array(p_nu, dtype=np.float64), np.array(p_u, dtype=np.float64)
    pot, g_nu, g_u = grad_fn(q_nu, q_u)
    h0 = pot + kinetic(p_nu, p_u, minv_nu, minv_u)
    for _ in range(n_steps):
        for i, b in enumerate(drifts):
            p_nu -= kicks[i] * eps * g_nu
            p_u -= kicks[i] * eps * g_u
            q_nu += b * eps * minv_nu * p_nu
            q_u += b * eps * minv_u * p_u
            pot, g_nu, g_u = grad_fn(q_nu, q_u)
        p_nu -= kicks[-1] * eps * g_nu
        p_u -= kicks[-1] * eps * g_u
    h1 = pot + kinetic(p_nu, p_u, minv_nu, minv_u)
    return q_nu, q_u, p_nu, p_u, h0, h1
