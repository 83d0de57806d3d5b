"""Leapfrog trajectories of the HIP library (graph-captured) against the FP64
oracle's leapfrog, and graph replay consistency."""
import numpy as np
import pytest

import fzw_inputs as fi
from oracle import hmc
from tests.helpers import fp32, mock_case

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from tests.gpu_helpers import dev, dev_counts, host, plan_for, relnorm  # noqa: E402


def _priors(w):
    mu, sig = [], []
    for regions, col in w.free:
        if col == fi.COL_BETA:
            mu.append(fi.PRIOR_MU_BETA), sig.append(fi.PRIOR_SIGMA_BETA)
        else:
            mu.append(fi.PRIOR_MU_ALPHA), sig.append(fi.PRIOR_SIGMA_ALPHA)
    return np.array(mu), np.array(sig)


def _tie(w):
    tie = -np.ones(w.n_regions * 4, dtype=int)
    for f, (regions, col) in enumerate(w.free):
        for r in regions:
            tie[r * 4 + col] = f
    return tie


def _setup(name, n):
    w, m, nu_t, nu_e, counts = mock_case(name, n)
    ch = w.chains[0]
    # every input as the float32 values the GPU is handed
    nu = fp32(fi.near_truth_noise(ch))
    mu, sig = _priors(w)
    u0 = fp32(np.log(np.array([ch.bias[r[0], c] for r, c in w.free])))
    g = fi.rng_for(ch, fi.ROLE_MOMENTUM)
    p_nu = fp32(g.standard_normal(nu.shape))
    p_u = fp32(g.standard_normal(u0.shape))
    return w, m, counts, nu, u0, p_nu, p_u, mu, sig


@pytest.mark.parametrize("scheme", ["leapfrog", "blanes2", "yoshida4"])
@pytest.mark.parametrize("case", [("c0fd", None), ("c2", 32)])
def test_leapfrog_matches_oracle(case, scheme):
    """A graph-captured trajectory of each splitting scheme against the
    oracle's integrator: H at both ends to 1e-6 relative, end state 1e-4."""
    name, n = case
    w, m, counts, nu, u0, p_nu, p_u, mu, sig = _setup(name, n)
    ch = w.chains[0]
    eps, steps = float(fp32(2e-3)), 4
    minv_u = fp32(np.full(u0.shape, 1e-2))
    bias = fp32(ch.bias)
    gfn = lambda q, u: hmc.potential_and_grad(m, q, u, bias, w.free, mu, sig, counts)
    q1, u1, p1, pu1, h0, h1 = hmc.integrate(gfn, nu, u0, p_nu, p_u, 1.0, minv_u, eps, steps, scheme)

    plan = plan_for(w)
    plan.set_counts(0, dev_counts(counts))
    plan.set_sampling(_tie(w), mu, sig)
    plan.set_integrator(scheme)
    t_nu, t_u = dev(nu.ravel()), dev(u0[None])
    t_p, t_pu = dev(p_nu.ravel()), dev(p_u[None])
    base = dev(bias[None])
    minv = torch.ones_like(t_nu)
    t_minv_u = dev(minv_u[None])
    step = dev(np.array([eps]))
    hs, he = plan.leapfrog(t_nu, t_u, t_p, t_pu, base, minv, t_minv_u, step, steps)
    g_h0, g_h1 = float(host(hs)[0]), float(host(he)[0])
    e_q = relnorm(host(t_nu).reshape(nu.shape) - nu, q1 - nu)
    e_p = relnorm(host(t_p).reshape(nu.shape), p1)
    e_u = float(np.max(np.abs(host(t_u)[0] - u1)))
    print(name, n, scheme, "H0 %.6e/%.6e H1 %.6e/%.6e dH gpu %.4e oracle %.4e  dq %.2e dp %.2e du %.2e" % (
        g_h0, h0, g_h1, h1, g_h1 - g_h0, h1 - h0, e_q, e_p, e_u))
    assert abs(g_h0 - h0) < 1e-6 * abs(h0)
    assert abs(g_h1 - h1) < 1e-6 * abs(h1)
    assert e_q < 1e-4 and e_p < 1e-4 and e_u < 1e-6


def test_graph_replay_matches_first_launch():
    """The trajectory graph is captured on the first call and replayed after:
    a replay from the same start state gives the same end state bit for bit,
    with eager work and synchronisation between the replays."""
    w, m, counts, nu, u0, p_nu, p_u, mu, sig = _setup("c0", None)
    ch = w.chains[0]
    plan = plan_for(w)
    plan.set_counts(0, dev_counts(counts))
    plan.set_sampling(_tie(w), mu, sig)
    bufs = [dev(nu.ravel()), dev(u0[None]), dev(p_nu.ravel()), dev(p_u[None])]
    start = [b.clone() for b in bufs]
    base = dev(ch.bias[None])
    minv = torch.ones_like(bufs[0])
    minv_u = dev(np.full((1, u0.size), 1e-2))
    step = dev(np.array([1e-3]))
    results = []
    for rep in range(3):
        for b, s0 in zip(bufs, start):
            b.copy_(s0)
        hs, he = plan.leapfrog(bufs[0], bufs[1], bufs[2], bufs[3], base, minv, minv_u, step, 3)
        torch.cuda.synchronize()
        results.append([b.clone() for b in bufs] + [hs.clone(), he.clone()])
        _ = (bufs[0] * 2).sum().item()      # eager work between replays
    for r in results[1:]:
        for a, b in zip(results[0], r):
            assert torch.equal(a, b)


def test_leapfrog_full_signed_table_matches_oracle():
    """All 64 entries of the 16-region table free (negative cut-off exponents
    as -exp(u), fzw_set_sampling_signs): a trajectory against the oracle's."""
    import dataclasses
    w, m, nu_t, nu_e, counts = mock_case("c2", 32)
    ch = w.chains[0]
    wf = dataclasses.replace(w, free=fi.full_table_free(w.n_regions))
    mu, sig = fi.prior_arrays(wf)
    u0 = fp32(fi.free_start(wf, ch))
    signs = fi.free_signs(wf, ch)
    nu = fp32(fi.near_truth_noise(ch))
    g = fi.rng_for(ch, fi.ROLE_MOMENTUM)
    p_nu = fp32(g.standard_normal(nu.shape))
    p_u = fp32(g.standard_normal(u0.shape))
    eps, steps = float(fp32(2e-3)), 4
    minv_u = fp32(np.full(u0.shape, 1e-3))
    bias = fp32(ch.bias)
    gfn = lambda q, u: hmc.potential_and_grad(m, q, u, bias, wf.free, mu, sig, counts, signs)
    q1, u1, p1, pu1, h0, h1 = hmc.leapfrog(gfn, nu, u0, p_nu, p_u, 1.0, minv_u, eps, steps)
    plan = plan_for(wf)
    plan.set_counts(0, dev_counts(counts))
    plan.set_sampling(fi.tie_array(wf), mu, sig)
    plan.set_sampling_signs(signs)
    t_nu, t_u = dev(nu.ravel()), dev(u0[None])
    t_p, t_pu = dev(p_nu.ravel()), dev(p_u[None])
    hs, he = plan.leapfrog(t_nu, t_u, t_p, t_pu, dev(bias[None]), torch.ones_like(t_nu), dev(minv_u[None]),
                           dev(np.array([eps])), steps)
    g_h0, g_h1 = float(host(hs)[0]), float(host(he)[0])
    e_q = relnorm(host(t_nu).reshape(nu.shape) - nu, q1 - nu)
    e_u = float(np.max(np.abs(host(t_u)[0] - u1)))
    print("64 free: H0 %.6e/%.6e H1 %.6e/%.6e dq %.2e du %.2e" % (g_h0, h0, g_h1, h1, e_q, e_u))
    assert abs(g_h0 - h0) < 1e-6 * abs(h0)
    assert abs(g_h1 - h1) < 1e-6 * abs(h1)
    assert e_q < 1e-4 and e_u < 1e-5
