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


# --------------------------------------------------------------------------
# Posterior-validation statistics (Section 4: power-spectrum monopole and
# quadrupole, reduced bispectrum as a function of the triangle's opening
# angle, cross-correlation coefficient and propagator).  Readings (the paper
# gives names, not formulas):
#   * multipoles with respect to a plane-parallel line of sight along z:
#     P_l(k) = (2l + 1) < P(k) L_l(mu) >_shell, mu = k_z / k;
#   * shells are [k_lo + i dk, k_lo + (i+1) dk); a half-spectrum mode with
#     0 < n_z < N/2 stands for itself and its mirror (weight 2);
#   * bispectrum by the FFT estimator over shells of width dk centred on
#     k1, k2 and k3 = sqrt(k1^2 + k2^2 + 2 k1 k2 cos theta), i.e. theta is the
#     angle between the wave vectors k1 and k2 (k3 = |k1 + k2|);
#     B = (dx^6 / N^3) sum_x I1 I2 I3 / sum_x J1 J2 J3 with I_i the inverse
#     DFT of delta_hat on shell i and J_i that of the shell's indicator;
#   * Q = B / (P1 P2 + P2 P3 + P3 P1) with P_i the monopole on the same shells;
#   * cross-correlation C(k) = P_ab / sqrt(P_aa P_bb); propagator
#     G(k) = P_ab / P_bb (b the reference field).

def _kgrid(n, box):
    kf = 2.0 * np.pi / box
    nf = np.fft.fftfreq(n, 1.0 / n)
    nz = np.fft.rfftfreq(n, 1.0 / n)
    kx, ky, kz = kf * nf[:, None, None], kf * nf[None, :, None], kf * nz[None, None, :]
    kmag = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    wt = np.where((nz > 0) & (nz < n / 2), 2.0, 1.0)[None, None, :] * np.ones_like(kmag)
    return kmag, kz, wt


def multipoles(a, b, box, k_lo, dk, nbins):
    """Monopole and quadrupole of the cross spectrum of real fields a, b
    (b = a for the auto spectrum).  Returns k_mean, modes, P0, P2 per bin."""
    n = a.shape[0]
    dx = box / n
    fa = np.fft.rfftn(a)
    fb = fa if b is None else np.fft.rfftn(b)
    pk = (dx ** 3 / n ** 3) * np.real(fa * np.conj(fb))
    kmag, kz, wt = _kgrid(n, box)
    with np.errstate(invalid="ignore", divide="ignore"):
        mu = np.where(kmag > 0, kz / kmag, 0.0)
    l2 = 0.5 * (3.0 * mu * mu - 1.0)
    idx = np.floor((kmag - k_lo) / dk).astype(np.int64).ravel()
    ok = (idx >= 0) & (idx < nbins) & (kmag.ravel() > 0)
    w = wt.ravel()[ok]
    cnt = np.bincount(idx[ok], weights=w, minlength=nbins)
    km = np.bincount(idx[ok], weights=(w * kmag.ravel()[ok]), minlength=nbins)
    p0 = np.bincount(idx[ok], weights=(w * pk.ravel()[ok]), minlength=nbins)
    p2 = np.bincount(idx[ok], weights=(w * (pk * l2).ravel()[ok]), minlength=nbins)
    with np.errstate(invalid="ignore", divide="ignore"):
        return km / cnt, cnt, p0 / cnt, 5.0 * p2 / cnt


def cross_statistics(a, ref, box, k_lo, dk, nbins):
    """Cross-correlation coefficient C(k) and propagator G(k) of a field with
    a reference field."""
    _, _, pab, _ = multipoles(a, ref, box, k_lo, dk, nbins)
    _, _, paa, _ = multipoles(a, None, box, k_lo, dk, nbins)
    _, _, pbb, _ = multipoles(ref, None, box, k_lo, dk, nbins)
    with np.errstate(invalid="ignore", divide="ignore"):
        return pab / np.sqrt(paa * pbb), pab / pbb


def _shell_field(spec, kmag, lo, hi, n):
    return np.fft.irfftn(np.where((kmag >= lo) & (kmag < hi), spec, 0.0), s=(n, n, n), axes=(0, 1, 2))


def bispectrum(delta, box, k1, k2, dk, thetas):
    """Bispectrum and reduced bispectrum for shells of width dk centred on k1,
    k2 and k3(theta).  Returns k3, B, Q and the number of triangles."""
    n = delta.shape[0]
    dx = box / n
    fd = np.fft.rfftn(delta)
    kmag, _, _ = _kgrid(n, box)
    ones = np.ones_like(fd)

    def shell(kc):
        lo, hi = kc - 0.5 * dk, kc + 0.5 * dk
        return _shell_field(fd, kmag, lo, hi, n), _shell_field(ones, kmag, lo, hi, n)

    def pmono(kc):
        sel = (kmag >= kc - 0.5 * dk) & (kmag < kc + 0.5 * dk)
        _, _, wt = _kgrid(n, box)
        pk = (dx ** 3 / n ** 3) * np.abs(fd) ** 2
        return float(np.sum(wt[sel] * pk[sel]) / np.sum(wt[sel]))

    i1, j1 = shell(k1)
    i2, j2 = shell(k2)
    p1, p2 = pmono(k1), pmono(k2)
    out_k3, out_b, out_q, out_t = [], [], [], []
    for th in thetas:
        k3 = float(np.sqrt(k1 * k1 + k2 * k2 + 2.0 * k1 * k2 * np.cos(th)))
        i3, j3 = shell(k3)
        tri = float(np.sum(j1 * j2 * j3))
        b = (dx ** 6 / n ** 3) * float(np.sum(i1 * i2 * i3)) / tri
        p3 = pmono(k3)
        out_k3.append(k3)
        out_b.append(b)
        out_q.append(b / (p1 * p2 + p2 * p3 + p3 * p1))
        out_t.append(tri * n ** 6)
    return np.array(out_k3), np.array(out_b), np.array(out_q), np.array(out_t)
