"""Helpers for the GPU parity tests: plans from workload descriptions, device
copies, and error metrics."""
import numpy as np
import torch

import fzw_inputs as fi


def plan_for(w, chains=None):
    from paper_2506_03969_amd import CosmoParams, Plan, WebParams
    c = w.cosmo
    cosmo = CosmoParams(c.omega_m, c.h, c.sigma8, c.n_s, c.d1, c.f_growth, c.r_s, c.rsd_axis, c.tau_sc,
                        c.x_floor)
    web = WebParams(tuple(w.web.kinds), tuple(w.web.smooth_r), tuple(w.web.ell), w.web.steepness,
                    w.web.lambda_th)
    chs = w.chains if chains is None else [w.chains[i] for i in chains]
    return Plan([ch.n for ch in chs], [ch.box for ch in chs], cosmo, web)


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def dev_counts(c):
    return torch.from_numpy(np.ascontiguousarray(c).astype(np.uint16).view(np.int16)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def relnorm(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm((x - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


def bias_entry_error(g, ref):
    """max |g - ref| / max(|ref|, 1e-3 max|ref|) over the table entries."""
    g = np.asarray(g, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    return float(np.max(np.abs(g - ref) / den))
