"""Wiener-filter starting point of the chains (oracle, FP64).

Test infrastructure only (see oracle/__init__.py).

Section 2.2 (initialisation): each chain starts from the observed tracer
contrast delta_tr = n N^3 / N_tr - 1, Wiener-filtered (Zaroubi et al. 1995)
with the linear power spectrum taken as known and peculiar motions ignored,
and mapped back to white noise.  Readings (the paper gives no formula):
  * the signal is the linear density delta_L = M_delta(nu) with nu ~ N(0, I),
    so its spectrum per rfft mode is N^3 h(k)^2 with h = sqrt(P/dx^3);
  * the noise is Poisson shot noise of the tracers, white with variance
    1/nbar per cell, nbar = N_tr / N^3;
  * the white-noise start is the posterior mean of nu given delta_tr under
    that linear Gaussian model, which is diagonal in Fourier space:
        nu_hat = h / (h^2 + 1/nbar) * rfftn(delta_tr),   nu_hat(k=0) = 0.
"""
from __future__ import annotations

import numpy as np


def tracer_contrast(counts):
    """delta_tr = n N^3 / N_tr - 1."""
    c = np.asarray(counts, dtype=np.float64)
    return c * (c.size / c.sum()) - 1.0


def wiener_white_noise(model, counts):
    """White-noise field whose linear density is the Wiener filter of the
    tracer contrast (module docstring)."""
    g = model.g
    d = tracer_contrast(counts)
    nbar = float(np.sum(counts)) / d.size
    h = model.hk
    filt = np.where(h > 0, h / (h * h + 1.0 / nbar), 0.0)
    return g.irfft(filt * g.rfft(d))
