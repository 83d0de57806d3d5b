"""Binned power-spectrum estimator (oracle, FP64; a test tool).

Test infrastructure only (see oracle/__init__.py).

With the Fourier convention of Appendix A (F = dx^3 times the unnormalised DFT),
P(k) = <|F delta|^2> / L^3 = (dx^3 / N^3) <|rfftn(delta)|^2>.
"""
from __future__ import annotations

import numpy as np


def power_spectrum(delta, box: float, edges):
    n = delta.shape[0]
    dx = box / n
    dk = np.fft.rfftn(delta)
    pk = (dx ** 3 / n ** 3) * np.abs(dk) ** 2
    kf = 2.0 * np.pi / box
    nf = np.fft.fftfreq(n, 1.0 / n)
    nz = np.fft.rfftfreq(n, 1.0 / n)
    kmag = kf * np.sqrt(nf[:, None, None] ** 2 + nf[None, :, None] ** 2 + nz[None, None, :] ** 2)
    # modes strictly inside the half axis stand for themselves and their mirror
    wt = np.where((nz > 0) & (nz < n / 2), 2.0, 1.0)[None, None, :] * np.ones_like(kmag)
    idx = np.digitize(kmag.ravel(), edges) - 1
    ok = (idx >= 0) & (idx < len(edges) - 1)
    num = np.bincount(idx[ok], weights=(pk * wt).ravel()[ok], minlength=len(edges) - 1)
    kw = np.bincount(idx[ok], weights=(kmag * wt).ravel()[ok], minlength=len(edges) - 1)
    cnt = np.bincount(idx[ok], weights=wt.ravel()[ok], minlength=len(edges) - 1)
    with np.errstate(invalid="ignore", divide="ignore"):
        return kw / cnt, num / cnt, cnt
