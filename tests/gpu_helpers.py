"""Helpers for the GPU parity tests: plans from workload descriptions, device
copies, and error metrics."""
import numpy as np
import torch

import fzw_inputs as fi


def plan_for(w, chains=None, checkpoint=False):
    from paper_2506_03969_amd import CosmoParams, Plan, WebParams
    c = w.cosmo
    cosmo = CosmoParams(c.omega_m, c.h, c.sigma8, c.n_s, c.d1, c.f_growth, c.r_s, c.rsd_axis, c.tau_sc,
                        c.x_floor)
    web = WebParams(tuple(w.web.kinds), tuple(w.web.smooth_r), tuple(w.web.ell), w.web.steepness,
                    w.web.lambda_th)
    chs = w.chains if chains is None else [w.chains[i] for i in chains]
    return Plan([ch.n for ch in chs], [ch.box for ch in chs], cosmo, web, checkpoint=checkpoint)


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def dev_counts(c):
    return torch.from_numpy(np.ascontiguousarray(c).astype(np.uint16).view(np.int16)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


from tests.helpers import bias_entry_error, relnorm  # noqa: E402,F401  (numpy-only metrics)
