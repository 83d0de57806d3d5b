"""Straight-line float64 PyTorch forward model used to cross-check the oracle's
hand-written adjoint with automatic differentiation (CPU only).

It re-implements only the differentiable operations (FFTs, products, CIC with
differentiable weights, symmetric eigenvalues, sigmoids, bias, NB likelihood);
the constant spectral filters are taken from the oracle model instance.
"""
import numpy as np
import torch


def logl_torch(m, nu, bias, counts):
    s, g = m.s, m.g
    n = s.n
    t = lambda a: torch.as_tensor(np.broadcast_to(a, np.broadcast(a, np.empty((n, n, n // 2 + 1))).shape).copy())
    hk, kern = t(m.hk), t(m.kern)
    kk = [t(k) for k in g.k]
    ko = [t(k) for k in g.k_odd]
    ik2 = t(g.inv_k2)
    rf = lambda x: torch.fft.rfftn(x)
    irf = lambda x: torch.fft.irfftn(x, s=(n, n, n))

    def hf(i, j):
        return kk[i] ** 2 if i == j else ko[i] * ko[j]

    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    dl_hat = hk * rf(nu)
    dl = irf(dl_hat)
    xx, yy, zz, xy, xz, yz = [irf(hf(i, j) * ik2 * dl_hat) for (i, j) in pairs]
    s2 = xx * yy + xx * zz + yy * zz - xy ** 2 - xz ** 2 - yz ** 2
    a = 1 - 2 * s.d1 * dl / 3
    if s.tau_sc > 0:
        hv = 0.5 * (a + torch.sqrt(a * a + s.tau_sc ** 2))
    else:
        hv = torch.clamp(a, min=0.0)
    dsc = 3 * (torch.sqrt(hv) - 1)
    q = kern * (s.d1 * dl_hat + (3 / 7) * s.d1 ** 2 * rf(s2)) - (1 - kern) * rf(dsc)
    psi = [irf(1j * ko[j] * ik2 * q) for j in range(3)]
    grid = torch.as_tensor(np.indices((n, n, n), dtype=np.float64))
    pos = [grid[j] + psi[j] / g.dx for j in range(3)]
    if s.rsd_axis == 3:
        # radial: move each particle along its ray from the box centre by the
        # line-of-sight component of f Psi
        ray = torch.stack(pos) - 0.5 * n
        dist = torch.sqrt(torch.sum(ray * ray, dim=0))
        rhat = ray / dist
        vlos = torch.sum(s.f_growth * torch.stack(psi) / g.dx * rhat, dim=0)
        pos = [pos[j] + vlos * rhat[j] for j in range(3)]
    elif s.rsd_axis >= 0:
        pos[s.rsd_axis] = pos[s.rsd_axis] + s.f_growth * psi[s.rsd_axis] / g.dx
    p = torch.stack([c.reshape(-1) for c in pos])
    base = torch.floor(p.detach())
    fr = p - base
    b = base.long() % n
    rho = torch.zeros(n ** 3, dtype=torch.float64)
    for ox in (0, 1):
        for oy in (0, 1):
            for oz in (0, 1):
                w = ((fr[0] if ox else 1 - fr[0]) * (fr[1] if oy else 1 - fr[1])
                     * (fr[2] if oz else 1 - fr[2]))
                idx = (((b[0] + ox) % n) * n + (b[1] + oy) % n) * n + (b[2] + oz) % n
                rho = rho.index_add(0, idx, w)
    rho = rho.reshape(n, n, n)
    delta = rho - 1
    dh = rf(delta)
    pws = []
    for mult in m.web_mult:
        mm = t(mult)
        comps = [irf(hf(i, j) * mm * dh).reshape(-1) for (i, j) in pairs]
        mat = torch.stack([torch.stack([comps[0], comps[3], comps[4]], -1),
                           torch.stack([comps[3], comps[1], comps[5]], -1),
                           torch.stack([comps[4], comps[5], comps[2]], -1)], -2)
        lam = torch.linalg.eigvalsh(mat).flip(-1)
        w = torch.sigmoid(s.steepness * (lam - s.lambda_th))
        pws.append(torch.stack([1 - w[:, 0], w[:, 0] - w[:, 1], w[:, 1] - w[:, 2], w[:, 2]]))
    if len(pws) == 1:
        preg = pws[0]
    else:
        preg = (pws[0][:, None, :] * pws[1][None, :, :]).reshape(16, -1)
    theta = bias.T @ preg
    al, ep, rh, be = theta
    x = torch.clamp(1 + delta.reshape(-1), min=s.x_floor)
    lnx = torch.log(x)
    logf = al * lnx - torch.exp(ep * (lnx - torch.log(rh)))
    cn = torch.as_tensor(np.asarray(counts, dtype=np.float64).reshape(-1))
    ntr = cn.sum()
    ln_nbar = torch.log(ntr) - torch.logsumexp(logf, 0) + logf
    nbar = torch.exp(ln_nbar)
    l1p = torch.log1p(nbar / be)
    lg = torch.lgamma(cn + be) - torch.lgamma(be) - torch.lgamma(cn + 1)
    ell = lg - (be + cn) * l1p + cn * (ln_nbar - torch.log(be))
    return ell.sum()


def value_and_grad_torch(m, nu, bias, counts):
    nu_t = torch.tensor(nu, dtype=torch.float64, requires_grad=True)
    b_t = torch.tensor(bias, dtype=torch.float64, requires_grad=True)
    v = logl_torch(m, nu_t, b_t, counts)
    v.backward()
    return float(v.detach()), nu_t.grad.numpy(), b_t.grad.numpy()
