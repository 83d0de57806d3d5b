"""Mock data from the forward model (oracle, FP64).

Test infrastructure only (see oracle/__init__.py).

Section 3 recipe: draw a truth white-noise field, run the forward model with the
truth bias, scale the mean field to the target mean count, then draw
lambda ~ Gamma(beta_i, nbar_i / beta_i) and n* ~ Poisson(lambda) (Section 2.7).
"""
from __future__ import annotations

import numpy as np


def make_counts(model, nu_truth, bias, mean_count, draw):
    """`draw(nbar, beta)` supplies the Gamma-Poisson random draw (seeded by the
    caller).  Returns (counts uint16 [N,N,N], nbar_truth float64 [N,N,N])."""
    st = model.forward(nu_truth, bias)
    f = st["f"]
    nbar = f * (mean_count * f.size / f.sum())
    beta = st["theta"][3]
    n = model.s.n
    counts = draw(nbar, beta)
    return counts.reshape(n, n, n), nbar.reshape(n, n, n)
