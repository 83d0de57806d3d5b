"""Forward model and hand-written adjoint (oracle, FP64).

Test infrastructure only (see oracle/__init__.py).

The forward model of Section 2.1 (Eq. 1) is the composition
    nbar = M_b( M_Psi( M_delta(nu) ), b )
followed by the negative-binomial likelihood of Section 2.7.  Each stage below
follows the passage named in its comment.  Spectral conventions (not stated in
the paper; fixed here and in the GPU library alike):
  * k_j = 2 pi n_j / L with n_j from the FFT frequency ordering; 1/k^2 := 0 at k=0;
  * a factor with an odd power of k_j is set to zero on that axis' Nyquist
    index, so every "rfft -> multiply -> irfft" stage is an exactly real-linear
    map whose adjoint is the same chain with the conjugate multiplier;
  * rfftn is unnormalised and irfftn carries 1/N^3 (numpy convention).

Readings where the paper is silent or garbled:
  * 2LPT: Psi = -D1 grad phi1 + D2 grad phi2, lap phi1 = delta_L,
    lap phi2 = sum_{i<j} (phi1_ii phi1_jj - phi1_ij^2), D2 = -3/7 D1^2.
  * spherical collapse: div Psi_SC = 3 (sqrt(max(1 - 2 D1 delta_L / 3, 0)) - 1),
    curl free; optional smooth hinge of width tau_sc.
  * ALPT kernel K(k) = exp(-k^2 r_s^2 / 2) on the 2LPT part, 1-K on the SC part.
  * particles start on the mesh nodes, one per cell; CIC onto the same nodes.
  * RSD: plane-parallel along z, s_z = x_z + f Psi_z; or radial about an
    observer at the box centre, s = x + f (Psi.r) r / |r|^2 with r = x - centre
    the particle's unwrapped Eulerian position, and no shift at r = 0.
  * Phi-web tensor k_i k_j W_G(kR)/k^2 delta_k; delta-web tensor
    ell^2 k_i k_j W_G(kR) delta_k ("parity unpinned": sign and scale reading).
  * eigenvalues sorted descending, memberships V,S,F,K = 1-w1, w1-w2, w2-w3, w3;
    16 regions are products of the two webs' memberships, index 4*j + k.
  * bias f = x^alpha exp(-(x/rho)^eps), x = max(1+delta, x_floor), signed eps
    (eps < 0 is the low-density cut-off) ("parity unpinned": sign reading).
  * all four bias parameters (alpha, eps, rho, beta) interpolated per voxel.
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np
import scipy.fft as sfft
from scipy import special

from . import cosmology

PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
RSD_RADIAL = 3          # rsd_axis value selecting radial RSD about the box centre
WEB_PHI, WEB_DELTA = 0, 1
# FFT threads: the host's thread share where one is set, else every core
_WORKERS = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1


def set_workers(n: int) -> None:
    global _WORKERS
    _WORKERS = max(1, int(n))


class Grid:
    """Periodic cubic mesh of N^3 cells and side L with its rfft wave vectors."""

    def __init__(self, n: int, box: float):
        self.n = int(n)
        self.box = float(box)
        self.dx = self.box / self.n
        kf = 2.0 * np.pi / self.box
        nf = np.fft.fftfreq(self.n, 1.0 / self.n)
        nz = np.fft.rfftfreq(self.n, 1.0 / self.n)
        self.k = [(kf * nf)[:, None, None], (kf * nf)[None, :, None], (kf * nz)[None, None, :]]
        nyq = self.n // 2 if self.n % 2 == 0 else None
        idx = [nf[:, None, None], nf[None, :, None], nz[None, None, :]]
        self.k_odd = []
        for j in range(3):
            if nyq is None:
                self.k_odd.append(self.k[j])
            else:
                self.k_odd.append(np.where(np.abs(idx[j]) == nyq, 0.0, self.k[j]))
        self.k2 = self.k[0] ** 2 + self.k[1] ** 2 + self.k[2] ** 2
        self.kmag = np.sqrt(self.k2)
        with np.errstate(divide="ignore"):
            self.inv_k2 = np.where(self.k2 > 0, 1.0 / np.where(self.k2 > 0, self.k2, 1.0), 0.0)

    def rfft(self, x):
        return sfft.rfftn(x, workers=_WORKERS)

    def irfft(self, x):
        return sfft.irfftn(x, s=(self.n,) * 3, workers=_WORKERS)

    def hessian_factor(self, i: int, j: int):
        """k_i k_j, with the odd-factor Nyquist rule for i != j."""
        if i == j:
            return self.k[i] ** 2
        return self.k_odd[i] * self.k_odd[j]


@dataclass
class Settings:
    """Plain numbers the oracle needs; built from the workload description."""
    n: int
    box: float
    omega_m: float
    h: float
    sigma8: float
    n_s: float
    d1: float
    f_growth: float
    r_s: float
    rsd_axis: int
    tau_sc: float
    x_floor: float
    web_kinds: tuple
    web_smooth: tuple
    web_ell: tuple
    steepness: float
    lambda_th: float

    @classmethod
    def from_workload(cls, cosmo, web, chain):
        return cls(chain.n, chain.box, cosmo.omega_m, cosmo.h, cosmo.sigma8, cosmo.n_s,
                   cosmo.d1, cosmo.f_growth, cosmo.r_s, cosmo.rsd_axis, cosmo.tau_sc,
                   cosmo.x_floor, tuple(web.kinds), tuple(web.smooth_r), tuple(web.ell),
                   web.steepness, web.lambda_th)

    @property
    def n_regions(self):
        return 4 ** len(self.web_kinds)


def nb_loglike(n, ln_nbar, beta):
    """Section 2.7: log-pmf of n under lambda ~ Gamma(shape beta, scale nbar/beta),
    n ~ Poisson(lambda), i.e. the negative binomial
      lnG(n+beta) - lnG(beta) - lnG(n+1) + beta ln(beta/(beta+nbar)) + n ln(nbar/(beta+nbar)),
    written with log1p so that it stays finite for tiny nbar.  Returns the
    log-pmf and log1p(nbar/beta)."""
    nbar = np.exp(ln_nbar)
    l1p = np.log1p(nbar / beta)
    lg = special.gammaln(n + beta) - special.gammaln(beta) - special.gammaln(n + 1.0)
    return lg - (beta + n) * l1p + n * (ln_nbar - np.log(beta)), l1p


def _sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


class Model:
    """The forward model on one mesh, with precomputed spectral filters."""

    def __init__(self, s: Settings, power_amplitude: float | None = None):
        self.s = s
        self.g = Grid(s.n, s.box)
        g = self.g
        self.amp = cosmology.power_amplitude(s) if power_amplitude is None else power_amplitude
        # Appendix A: white-noise filter h(k) = sqrt(P(k)/dx^3), h(0)=0.
        self.hk = cosmology.white_noise_filter(g.kmag, g.dx, s, self.amp)
        # Section 2.3: ALPT Gaussian kernel of radius r_s.
        self.kern = np.exp(-0.5 * g.k2 * s.r_s ** 2)
        # Section 2.8: radial part of each web's tensor multiplier.
        self.web_mult = []
        for kind, r, ell in zip(s.web_kinds, s.web_smooth, s.web_ell):
            wg = np.exp(-0.5 * g.k2 * r * r)
            if kind == WEB_PHI:
                self.web_mult.append(wg * g.inv_k2)
            else:
                self.web_mult.append(ell * ell * wg)

    # ------------------------------------------------------------------ stages
    def linear_density_hat(self, nu):
        """Appendix A: delta_L spectrum = h(k) rfftn(nu)."""
        return self.hk * self.g.rfft(nu)

    def hinge(self, a):
        tau = self.s.tau_sc
        if tau > 0:
            r = np.sqrt(a * a + tau * tau)
            return 0.5 * (a + r), 0.5 * (1.0 + a / r)
        return np.maximum(a, 0.0), (a > 0).astype(np.float64)

    def alpt(self, dl_hat):
        """Section 2.3: Psi = K o Psi_2LPT + (1-K) o Psi_SC.  Returns Psi (3,N,N,N)
        and the intermediates the adjoint needs."""
        g, s = self.g, self.s
        d1 = s.d1
        dl = g.irfft(dl_hat)
        phi = [g.irfft(g.hessian_factor(i, j) * g.inv_k2 * dl_hat) for (i, j) in PAIRS]
        xx, yy, zz, xy, xz, yz = phi
        s2 = xx * yy + xx * zz + yy * zz - xy * xy - xz * xz - yz * yz
        a = 1.0 - 2.0 * d1 * dl / 3.0
        hv, _ = self.hinge(a)
        dsc = 3.0 * (np.sqrt(hv) - 1.0)
        q_hat = (self.kern * (d1 * dl_hat + (3.0 / 7.0) * d1 * d1 * g.rfft(s2))
                 - (1.0 - self.kern) * g.rfft(dsc))
        psi = np.stack([g.irfft(1j * g.k_odd[j] * g.inv_k2 * q_hat) for j in range(3)])
        return psi, dict(dl=dl, phi=phi, s2=s2, a=a, dsc=dsc)

    def radial_frame(self, psi):
        """Section 2.9 with the observer at the box centre (cell units): the
        line-of-sight vector r from the observer to the real-space position,
        |r|^2, the velocity displacement u = f Psi / dx (b_v = 1), and the
        coefficient a = (u.r)/|r|^2 of the shift a r (0 where r = 0)."""
        n, dx = self.s.n, self.g.dx
        grid = np.indices((n, n, n), dtype=np.float64)
        r = grid + psi / dx - 0.5 * n
        r2 = np.sum(r * r, axis=0)
        u = self.s.f_growth * psi / dx
        safe = np.where(r2 > 0, r2, 1.0)
        a = np.where(r2 > 0, np.sum(u * r, axis=0) / safe, 0.0)
        return r, r2, u, a

    def positions(self, psi):
        """Particle positions in cell units (lattice node + displacement), in
        redshift space where RSD is on (Section 2.9): plane-parallel along the
        configured axis, or radial about the box centre."""
        n, dx = self.s.n, self.g.dx
        grid = np.indices((n, n, n), dtype=np.float64)
        pos = grid + psi / dx
        if self.s.rsd_axis == RSD_RADIAL:
            r, _, _, a = self.radial_frame(psi)
            pos = pos + a * r
        elif self.s.rsd_axis >= 0:
            ax = self.s.rsd_axis
            pos[ax] = pos[ax] + self.s.f_growth * psi[ax] / dx
        return pos

    def cic(self, pos):
        """Cloud-in-cell assignment of unit-mass particles; returns rho (mean 1)."""
        n = self.s.n
        p = pos.reshape(3, -1)
        base = np.floor(p)
        t = p - base
        b = base.astype(np.int64) % n
        rho = np.zeros(n ** 3)
        for ox in (0, 1):
            wx = t[0] if ox else 1.0 - t[0]
            ix = (b[0] + ox) % n
            for oy in (0, 1):
                wy = t[1] if oy else 1.0 - t[1]
                iy = (b[1] + oy) % n
                for oz in (0, 1):
                    wz = t[2] if oz else 1.0 - t[2]
                    iz = (b[2] + oz) % n
                    rho += np.bincount((ix * n + iy) * n + iz, weights=wx * wy * wz,
                                       minlength=n ** 3)
        return rho.reshape(n, n, n)

    def cic_adjoint(self, pos, drho):
        """Adjoint of `cic` with respect to the positions (right-sided derivative
        at cell faces)."""
        n = self.s.n
        p = pos.reshape(3, -1)
        base = np.floor(p)
        t = p - base
        b = base.astype(np.int64) % n
        dr = drho.reshape(-1)
        out = np.zeros_like(p)
        for ox in (0, 1):
            wx, gx = (t[0], 1.0) if ox else (1.0 - t[0], -1.0)
            ix = (b[0] + ox) % n
            for oy in (0, 1):
                wy, gy = (t[1], 1.0) if oy else (1.0 - t[1], -1.0)
                iy = (b[1] + oy) % n
                for oz in (0, 1):
                    wz, gz = (t[2], 1.0) if oz else (1.0 - t[2], -1.0)
                    iz = (b[2] + oz) % n
                    v = dr[(ix * n + iy) * n + iz]
                    out[0] += v * gx * wy * wz
                    out[1] += v * wx * gy * wz
                    out[2] += v * wx * wy * gz
        return out.reshape(3, n, n, n)

    def web_tensors(self, delta_hat):
        """Section 2.8 / Appendix B: per web, the 6 unique components of the
        tensor (order xx, yy, zz, xy, xz, yz)."""
        g = self.g
        return [[g.irfft(g.hessian_factor(i, j) * m * delta_hat) for (i, j) in PAIRS]
                for m in self.web_mult]

    @staticmethod
    def _matrix(t6):
        xx, yy, zz, xy, xz, yz = [c.reshape(-1) for c in t6]
        m = np.empty((xx.size, 3, 3))
        m[:, 0, 0], m[:, 1, 1], m[:, 2, 2] = xx, yy, zz
        m[:, 0, 1] = m[:, 1, 0] = xy
        m[:, 0, 2] = m[:, 2, 0] = xz
        m[:, 1, 2] = m[:, 2, 1] = yz
        return m

    def eigen(self, t6, vectors=False):
        """Eigenvalues sorted descending (Appendix B ordering) and, optionally,
        the matching unit eigenvectors as columns."""
        m = self._matrix(t6)
        if vectors:
            w, v = np.linalg.eigh(m)
            return w[:, ::-1], v[:, :, ::-1]
        return np.linalg.eigvalsh(m)[:, ::-1], None

    def memberships(self, lam):
        """Eq. 'sigmoid' and Eq. 'soft_cweb_p': w_n = sigma(s (lam_n - lam_th));
        p = (V, S, F, K) = (1-w1, w1-w2, w2-w3, w3)."""
        w = _sigmoid(self.s.steepness * (lam - self.s.lambda_th))
        p = np.stack([1.0 - w[:, 0], w[:, 0] - w[:, 1], w[:, 1] - w[:, 2], w[:, 2]])
        return w, p

    @staticmethod
    def regions(p_webs):
        """One web: its 4 memberships.  Two webs: the 16 products p_j^Phi p_k^delta
        (region index 4*j + k)."""
        if len(p_webs) == 1:
            return p_webs[0]
        pa, pb = p_webs
        return (pa[:, None, :] * pb[None, :, :]).reshape(16, -1)

    # ------------------------------------------------------- web and bias
    def web_bias(self, delta, bias):
        """Section 2.8 and Eq. 'local_bias' on a density contrast delta: web
        tensors, sorted eigenvalues, sigmoid weights and memberships, region
        probabilities, per-voxel parameters interpolated over the regions
        (boxed equation of Section 2.8: the parameters, not the bias values,
        are mixed) and the unnormalised bias f.  Returns the intermediates."""
        s, g = self.s, self.g
        bias = np.asarray(bias, dtype=np.float64)
        tens = self.web_tensors(g.rfft(delta))
        lams, ws, ps = [], [], []
        for t6 in tens:
            lam, _ = self.eigen(t6)
            w, p = self.memberships(lam)
            lams.append(lam), ws.append(w), ps.append(p)
        preg = self.regions(ps)                     # [R, M]
        theta = bias.T @ preg                       # [4, M]: alpha, eps, rho, beta
        alpha, eps, rho_th, beta = theta
        d = np.asarray(delta).reshape(-1)
        x = np.maximum(1.0 + d, s.x_floor)
        lnx = np.log(x)
        ell_ = lnx - np.log(rho_th)
        u = np.exp(eps * ell_)
        logf = alpha * lnx - u                      # Eq. 'local_bias' (signed eps)
        f = np.exp(logf)
        return dict(tens=tens, lams=lams, ws=ws, ps=ps, preg=preg, theta=theta, x=x, lnx=lnx,
                    ellr=ell_, u=u, logf=logf, f=f)

    # ----------------------------------------------------------------- forward
    def forward(self, nu, bias, counts=None):
        """Run the forward model.  Returns a dict with every intermediate; when
        counts are given it also holds logL (Section 2.7, Eq. 'log_likelihood')."""
        s, g = self.s, self.g
        bias = np.asarray(bias, dtype=np.float64)
        st = {}
        dl_hat = self.linear_density_hat(nu)
        psi, lpt = self.alpt(dl_hat)
        pos = self.positions(psi)
        rho = self.cic(pos)
        delta = rho - 1.0
        st.update(nu=nu, bias=bias, dl_hat=dl_hat, psi=psi, pos=pos, rho=rho, delta=delta, **lpt)
        st.update(self.web_bias(delta, bias))
        theta = st["theta"]
        beta = theta[3]
        f, logf = st["f"], st["logf"]
        if counts is not None:
            n = np.asarray(counts, dtype=np.float64).reshape(-1)
            ntr = n.sum()
            sumf = f.sum()
            lnc = np.log(ntr) - np.log(sumf)        # C = N_tr / sum f (Eq. 'local_bias')
            ln_nbar = lnc + logf
            nbar = np.exp(ln_nbar)
            ell, l1p = nb_loglike(n, ln_nbar, beta)
            st.update(counts=n, ntr=ntr, sumf=sumf, lnc=lnc, nbar=nbar, l1p=l1p, ell=ell,
                      logl=float(ell.sum()))
        return st

    def nbar(self, st):
        return st["nbar"].reshape((self.s.n,) * 3)

    # ----------------------------------------------------------------- adjoint
    def value_and_grad(self, nu, bias, counts):
        st = self.forward(nu, bias, counts)
        dnu, dbias = self.adjoint(st)
        return st["logl"], dnu, dbias

    def adjoint(self, st):
        """Hand-written reverse pass: d logL / d nu and d logL / d bias table.
        Also records in `st` the cotangents of two intermediates: d logL /
        d rho ('drho', the density) and d logL / d Psi ('dpsi', the
        displacement, per particle)."""
        s, g = self.s, self.g
        n = st["counts"]
        alpha, eps, rho_th, beta = st["theta"]
        nbar, ntr = st["nbar"], st["ntr"]
        # likelihood: ghat = nbar dl/dnbar, normalisation C = N_tr / sum f
        ghat = beta * (n - nbar) / (beta + nbar)
        big_g = ghat.sum()
        af = ghat - big_g * nbar / ntr              # f * dlogL/df
        dbeta = (special.digamma(n + beta) - special.digamma(beta) - st["l1p"]
                 + (nbar - n) / (beta + nbar))
        u, lnx, ellr, x = st["u"], st["lnx"], st["ellr"], st["x"]
        dalpha = af * lnx
        deps = -af * u * ellr
        drho = af * u * eps / rho_th
        dtheta = np.stack([dalpha, deps, drho, dbeta])   # [4, M]
        d = st["delta"].reshape(-1)
        dx_direct = af * (alpha - eps * u) / x
        dx_direct = np.where(1.0 + d > s.x_floor, dx_direct, 0.0)
        preg = st["preg"]
        dbias = preg @ dtheta.T                     # [R, 4]
        # the sums of the magnitudes of each entry's per-voxel terms: the
        # scale of the rounding error of any evaluation that rounds the terms
        st["dbias_abs"] = np.abs(preg) @ np.abs(dtheta).T
        dp = st["bias"] @ dtheta                    # [R, M]
        ps = st["ps"]
        if len(ps) == 1:
            dps = [dp]
        else:
            d16 = dp.reshape(4, 4, -1)
            dps = [np.einsum("jkm,km->jm", d16, ps[1]), np.einsum("jkm,jm->km", d16, ps[0])]
        ddelta_hat = 0.0
        for wi, (t6, dpw) in enumerate(zip(st["tens"], dps)):
            w = st["ws"][wi]
            dw = np.stack([dpw[1] - dpw[0], dpw[2] - dpw[1], dpw[3] - dpw[2]], axis=1)
            dlam = dw * s.steepness * w * (1.0 - w)
            _, v = self.eigen(t6, vectors=True)
            dmat = np.einsum("mn,min,mjn->mij", dlam, v, v)
            comps = []
            for (i, j) in PAIRS:
                c = dmat[:, i, j] if i == j else 2.0 * dmat[:, i, j]
                comps.append(c.reshape((s.n,) * 3))
            m = self.web_mult[wi]
            for (i, j), c in zip(PAIRS, comps):
                ddelta_hat = ddelta_hat + g.hessian_factor(i, j) * m * g.rfft(c)
        ddelta = g.irfft(ddelta_hat) + dx_direct.reshape((s.n,) * 3)
        st["drho"] = ddelta
        # CIC adjoint, then the RSD chain rule
        dpos = self.cic_adjoint(st["pos"], ddelta)
        if s.rsd_axis == RSD_RADIAL:
            # s = x + a r, with x = q + psi, r = x - centre, u = f psi and
            # a = (u.r)/|r|^2: ds_i/dpsi_j = (1+a) delta_ij
            #   + r_i (u_j + (f - 2a) r_j) / |r|^2, transposed onto dpos
            r, r2, u, a = self.radial_frame(st["psi"])
            gr = np.where(r2 > 0, np.sum(dpos * r, axis=0) / np.where(r2 > 0, r2, 1.0), 0.0)
            dpos = (1.0 + a) * dpos + gr * (u + (s.f_growth - 2.0 * a) * r)
        dpsi = dpos / g.dx
        if 0 <= s.rsd_axis < 3:
            # s_ax = q_ax + (1+f) Psi_ax / dx
            dpsi[s.rsd_axis] = dpsi[s.rsd_axis] * (1.0 + s.f_growth)
        st["dpsi"] = dpsi
        # ALPT adjoint: conjugate multipliers
        dq_hat = 0.0
        for j in range(3):
            dq_hat = dq_hat + (-1j) * g.k_odd[j] * g.inv_k2 * g.rfft(dpsi[j])
        d1 = s.d1
        ds2 = g.irfft((3.0 / 7.0) * d1 * d1 * self.kern * dq_hat)
        ddsc = g.irfft(-(1.0 - self.kern) * dq_hat)
        dnu_hat = self.hk * d1 * self.kern * dq_hat
        hv, hd = self.hinge(st["a"])
        with np.errstate(divide="ignore", invalid="ignore"):
            ddl = np.where(hv > 0, -ddsc * d1 * hd / np.sqrt(np.where(hv > 0, hv, 1.0)), 0.0)
        xx, yy, zz, xy, xz, yz = st["phi"]
        dphi = [ds2 * (yy + zz), ds2 * (xx + zz), ds2 * (xx + yy),
                -2.0 * ds2 * xy, -2.0 * ds2 * xz, -2.0 * ds2 * yz]
        acc = g.rfft(ddl)
        for (i, j), c in zip(PAIRS, dphi):
            acc = acc + g.hessian_factor(i, j) * g.inv_k2 * g.rfft(c)
        dnu_hat = dnu_hat + self.hk * acc
        dnu = g.irfft(dnu_hat)
        return dnu, dbias
