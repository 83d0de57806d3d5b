"""No-U-turn transitions of the HIP library (fzw_nuts) against the FP64
oracle's transition on the same momentum and uniform draws, lock-step
batches against single chains, and the warm-up helpers.

A transition is a chain of random and sign decisions taken on energies and
momentum sums that the FP32 path and the FP64 oracle compute with different
rounding.  For every draw the oracle reports how far its closest decision
was from flipping, and it is also run three times with its gradients
perturbed at relative 1e-6 (the size of the FP32 path's gradient error) and
its particle positions at relative 2^-23 (the rounding of a position held in
float32).  The second matters on long trajectories: where a particle sits
within that rounding of a cell face at some leaf, the two paths may put it on
different sides, its cloud-in-cell derivative jumps, and the rest of the
trajectory can end elsewhere (a depth-7 tree at 16^3 passes such states at
most leaves).  Draws whose closest decision is nearer than the two paths'
expected difference (1e-3 in probability, 1e-3 relative in a U-turn dot
product), or whose perturbed oracle runs disagree on the tree or on the
potential of the new state, are not compared; the test needs at least three
compared draws per case.  Compared: the tree depth, the leapfrog steps
and the divergence flag exactly; the potential at the new state within 1e-5;
the acceptance statistic within 5e-3 plus the spread of the perturbed oracle
runs (a leaf whose energy sits on a steep stretch of the potential, such as a
tracer in a nearly empty cell, moves it by a few 1e-2; a particle within
FP32 rounding of a cell face at some leaf changes that leaf's gradient and
the rest of the trajectory at the 1e-4 level, which moves it by a few 1e-3);
the displacement of
the new state within 1e-3 normwise (bit-exact when the start point is
kept)."""
import copy
import dataclasses

import numpy as np
import pytest

import fzw_inputs as fi
from oracle import hmc, nuts
from tests.helpers import mock_case

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from tests.gpu_helpers import dev, dev_counts, host, plan_for, relnorm  # noqa: E402
from tests.test_gpu_hmc import _priors, _tie  # noqa: E402


def _draws(ch, seed, size, md):
    g = np.random.default_rng(np.random.SeedSequence([*ch.seed_key, fi.ROLE_MISC, seed]))
    z = g.standard_normal(size).astype(np.float32)
    uni = g.uniform(size=nuts.n_uniforms(md)).astype(np.float32)
    return z, uni


def _jittered(m, rng, rel):
    """A copy of the oracle model whose particle positions carry a fresh
    uniform error of up to `rel` relative (at least `rel` cells) at every
    evaluation."""
    mj = copy.copy(m)

    def positions(psi):
        pos = type(m).positions(mj, psi)
        return pos + rel * np.maximum(np.abs(pos), 1.0) * rng.uniform(-1.0, 1.0, pos.shape)
    mj.positions = positions
    return mj


POS_JITTER = 2.0 ** -23


def _oracle_potential(m, w, ch, mu, sig, counts, shape, noise=0.0, seed=0):
    """Potential and gradient of the oracle; with `noise`, the gradient is
    perturbed at that relative size and the particle positions at relative
    POS_JITTER (seeded)."""
    nv = int(np.prod(shape))
    rng = np.random.default_rng(seed)
    if noise:
        m = _jittered(m, rng, POS_JITTER)

    def pg(q):
        pot, gnu, gu = hmc.potential_and_grad(m, q[:nv].reshape(shape), q[nv:], ch.bias, w.free, mu, sig, counts)
        g = np.concatenate([gnu.ravel(), gu])
        if noise:
            g = g * (1.0 + noise * rng.standard_normal(g.size))
        return pot, g
    return pg


# (workload, mesh, step, max depth, draws): trees that reach the depth limit,
# trees that turn (depth 7 of 8), trajectories that diverge, and the two-web
# model.  Steps near the stability limit of the stiffest modes (0.1 here)
# make the trajectory itself chaotic: a 1e-6 change of the gradient then
# moves late leaves' energies by O(1), so they are not used.
CASES = [("c0fd", None, 0.03, 4, 12, "leapfrog"), ("c0fd", None, 0.04, 8, 12, "leapfrog"),
         ("c0fd", None, 0.3, 5, 8, "leapfrog"), ("c2", 32, 0.004, 4, 6, "leapfrog"),
         ("c0fd", None, 0.05, 4, 8, "blanes2"), ("c0fd", None, 0.05, 4, 6, "yoshida4")]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-%s-eps%g-d%d-%s" % (c[:4] + c[5:]))
def test_transition_matches_oracle(case):
    name, n, eps, md, n_draws, scheme = case
    w, m, nu_t, nu_e, counts = mock_case(name, n)
    ch = w.chains[0]
    mu, sig = _priors(w)
    nu0 = fi.near_truth_noise(ch).astype(np.float32)
    u0 = np.log(np.array([ch.bias[r[0], c] for r, c in w.free])).astype(np.float32)
    nv = nu0.size
    minv_u = np.full(u0.shape, 1e-2, dtype=np.float32)
    minv = np.concatenate([np.ones(nv), minv_u.astype(np.float64)])
    q0 = np.concatenate([nu0.ravel(), u0]).astype(np.float64)
    pg = _oracle_potential(m, w, ch, mu, sig, counts, nu0.shape)
    start = pg(q0)

    plan = plan_for(w)
    plan.set_counts(0, dev_counts(counts))
    plan.set_sampling(_tie(w), mu, sig)
    plan.set_integrator(scheme)
    base = dev(ch.bias[None])
    t_minv = torch.ones(nv, dtype=torch.float32, device="cuda")
    t_minv_u = dev(minv_u[None])
    step = dev(np.array([eps], dtype=np.float32))
    compared = 0
    for seed in range(n_draws):
        z, uni = _draws(ch, seed, q0.size, md)
        ref = nuts.transition(pg, q0, z.astype(np.float64), minv, eps, uni.astype(np.float64), md, start=start,
                              scheme=scheme)
        alts = [nuts.transition(_oracle_potential(m, w, ch, mu, sig, counts, nu0.shape, 1e-6, 100 * seed + v), q0,
                                z.astype(np.float64), minv, eps, uni.astype(np.float64), md, start=start,
                                scheme=scheme)
                for v in range(3)]
        robust = all((a.depth, a.n_leapfrog, a.diverging) == (ref.depth, ref.n_leapfrog, ref.diverging)
                     and abs(a.potential - ref.potential) < 1e-6 * abs(ref.potential) for a in alts)
        spread = max(abs(a.accept_stat - ref.accept_stat) for a in alts)
        t_nu, t_u = dev(nu0.ravel()), dev(u0[None])
        pot, acc, stats = plan.nuts(t_nu, t_u, dev(z[:nv]), dev(z[nv:][None]), base, t_minv, t_minv_u, step,
                                    dev(uni[None]), md)
        got_q = np.concatenate([host(t_nu).ravel(), host(t_u).ravel()])
        st = host(stats)[0]
        moved = not np.array_equal(ref.q, q0)
        e_q = relnorm(got_q - q0, ref.q - q0) if moved else float(np.max(np.abs(got_q - q0)))
        print("%s seed %d: depth %d/%d leaves %d/%d div %d/%d  U %.8e/%.8e  acc %.5f/%.5f  dq %.2e  "
              "margins choice %.3g turn %.3g, perturbed oracle %s, acc spread %.2g" % (
                  name, seed, st[0], ref.depth, st[1], ref.n_leapfrog, st[2], ref.diverging, float(host(pot)[0]),
                  ref.potential, float(host(acc)[0]), ref.accept_stat, e_q, ref.margin_choice, ref.margin_turn,
                  "agrees" if robust else "differs", spread))
        if ref.margin_choice < 1e-3 or ref.margin_turn < 1e-3 or not robust:
            continue
        compared += 1
        assert (int(st[0]), int(st[1]), bool(st[2])) == (ref.depth, ref.n_leapfrog, ref.diverging)
        assert abs(float(host(pot)[0]) - ref.potential) < 1e-5 * abs(ref.potential)
        assert abs(float(host(acc)[0]) - ref.accept_stat) < 5e-3 + 2 * spread
        if moved:
            assert e_q < 1e-3
        else:
            assert e_q == 0.0
    assert compared >= 3


def test_lock_step_batch_equals_single_chains():
    """Three chains of two mesh sizes in one plan give, bit for bit, what each
    gives alone, although their trajectories end after different doublings."""
    w = fi.workload("c0")
    chains = [fi.Chain(16, 125.0, w.chains[0].bias, 0.5, (7, 0)), fi.Chain(32, 250.0, w.chains[0].bias, 0.5, (7, 1)),
              fi.Chain(16, 125.0, w.chains[0].bias, 0.5, (7, 2))]
    ww = dataclasses.replace(w, chains=chains)
    mu, sig = _priors(ww)
    md = 5
    rng = np.random.default_rng(9)
    cnts = [rng.poisson(0.5, size=(c.n,) * 3).astype(np.uint16) for c in chains]
    nus = [fi.white_noise(c, fi.ROLE_EVAL_NU).astype(np.float32) for c in chains]
    nf = len(ww.free)
    us = [np.log(np.array([c.bias[r[0], col] for r, col in ww.free])).astype(np.float32) for c in chains]
    zs = [rng.standard_normal(c.n ** 3).astype(np.float32) for c in chains]
    zus = [rng.standard_normal(nf).astype(np.float32) for c in chains]
    unis = [rng.uniform(size=nuts.n_uniforms(md)).astype(np.float32) for c in chains]
    eps = np.array([0.05, 0.02, 0.2], dtype=np.float32)

    def run(sel):
        sub = dataclasses.replace(ww, chains=[chains[i] for i in sel])
        p = plan_for(sub)
        for k, i in enumerate(sel):
            p.set_counts(k, dev_counts(cnts[i]))
        p.set_sampling(_tie(sub), mu, sig)
        t_nu = dev(np.concatenate([nus[i].ravel() for i in sel]))
        t_u = dev(np.stack([us[i] for i in sel]))
        z = dev(np.concatenate([zs[i] for i in sel]))
        zu = dev(np.stack([zus[i] for i in sel]))
        base = dev(np.stack([chains[i].bias for i in sel]))
        minv = torch.ones_like(t_nu)
        minv_u = torch.full_like(t_u, 1e-2)
        uni = dev(np.stack([unis[i] for i in sel]))
        pot, acc, st = p.nuts(t_nu, t_u, z, zu, base, minv, minv_u, dev(eps[list(sel)]), uni, md)
        offs = [p.offsets[k] for k in range(len(sel))]
        return [(t_nu[offs[k]:offs[k] + chains[i].n ** 3].clone(), t_u[k].clone(), pot[k].clone(), acc[k].clone(),
                 st[k].clone()) for k, i in enumerate(sel)]

    together = run([0, 1, 2])
    depths = [int(r[4][0]) for r in together]
    print("depths", depths, "leaves", [int(r[4][1]) for r in together])
    for i in range(3):
        alone = run([i])[0]
        for a, b in zip(together[i], alone):
            assert torch.equal(a, b)
    assert len(set(int(r[4][1]) for r in together)) > 1     # the chains did stop at different points


def test_welford_and_inverse_mass_match_numpy():
    w = fi.small_variant(fi.workload("c0"), 16)
    p = plan_for(w)
    rng = np.random.default_rng(1)
    x = (rng.standard_normal((40, 5000)) * rng.uniform(0.2, 3.0, 5000) + 1.5).astype(np.float32)
    mean = torch.zeros(5000, dtype=torch.float32, device="cuda")
    m2 = torch.zeros_like(mean)
    for i, row in enumerate(x):
        p.welford(dev(row), mean, m2, i + 1)
    minv = torch.empty_like(mean)
    p.inverse_mass(m2, minv, len(x))
    n = len(x)
    var = x.astype(np.float64).var(0, ddof=1)
    want = n / (n + 5.0) * var + 1e-3 * 5.0 / (n + 5.0)
    assert np.allclose(host(mean), x.astype(np.float64).mean(0), rtol=1e-5, atol=1e-5)
    assert np.allclose(host(minv), want, rtol=1e-4)


def test_warmup_adapts_the_step_size():
    """A short warm-up on the 16^3 case: dual averaging moves the step towards
    a mean acceptance of 0.8 from a step that is far too large."""
    from paper_2506_03969_amd import DualAveraging
    w, m, nu_t, nu_e, counts = mock_case("c0fd")
    ch = w.chains[0]
    mu, sig = _priors(w)
    plan = plan_for(w)
    plan.set_counts(0, dev_counts(counts))
    plan.set_sampling(_tie(w), mu, sig)
    t_nu = dev(fi.near_truth_noise(ch).astype(np.float32).ravel())
    t_u = dev(np.log(np.array([ch.bias[r[0], c] for r, c in w.free]))[None].astype(np.float32))
    base = dev(ch.bias[None])
    minv = torch.ones_like(t_nu)
    minv_u = torch.full_like(t_u, 1e-2)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    md = 6
    da = DualAveraging(0.5)
    eps = 0.5
    accs = []
    for it in range(40):
        z = torch.randn(t_nu.numel(), generator=gen, device="cuda")
        zu = torch.randn(t_u.shape, generator=gen, device="cuda")
        uni = torch.rand((1, nuts.n_uniforms(md)), generator=gen, device="cuda")
        pot, acc, st = plan.nuts(t_nu, t_u, z, zu, base, minv, minv_u, dev(np.array([eps], dtype=np.float32)), uni, md)
        accs.append(float(host(acc)[0]))
        eps = da.update(accs[-1])
        assert np.isfinite(float(host(pot)[0]))
    print("eps final %.4f, mean accept of the last 10: %.3f" % (da.final(), np.mean(accs[-10:])))
    assert da.final() < 0.2
    assert np.mean(accs[-10:]) > 0.3
