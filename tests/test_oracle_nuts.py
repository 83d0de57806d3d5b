"""The oracle's NUTS transition and warm-up adaptation, pinned to what the
mathematics fixes: invariance of a Gaussian target, the one-leaf case as a
Metropolis-adjusted leapfrog step, the recursive formulation of the tree's
stopping rule, and the fixed points of dual averaging and Welford."""
import math

import numpy as np
import pytest

import fzw_inputs as fi
from oracle import hmc, nuts
from tests.helpers import mock_case

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _gaussian(cov):
    prec = np.linalg.inv(cov)
    return lambda q: (0.5 * float(q @ prec @ q), prec @ q)


def test_samples_keep_a_correlated_gaussian_invariant():
    """6000 transitions on a 3-D Gaussian with scales 0.4..3 and correlation
    0.6: sample mean and covariance within a few Monte Carlo errors."""
    a = np.diag([0.4, 1.0, 3.0])
    corr = np.array([[1.0, 0.6, 0.0], [0.6, 1.0, 0.3], [0.0, 0.3, 1.0]])
    cov = a @ corr @ a
    pg = _gaussian(cov)
    rng = np.random.default_rng(11)
    q = np.zeros(3)
    start = pg(q)
    draws, depths = [], []
    md = 6
    for it in range(6000):
        t = nuts.transition(pg, q, rng.standard_normal(3), 1.0, 0.25,
                            rng.uniform(size=nuts.n_uniforms(md)), md, start=start)
        q, start = t.q, (t.potential, t.grad)
        draws.append(q)
        depths.append(t.depth)
    x = np.array(draws[500:])
    se = np.sqrt(np.diag(cov) / len(x))
    assert np.all(np.abs(x.mean(0)) < 6 * se * 3)      # allow an autocorrelation time of ~9
    c = np.cov(x.T)
    assert np.allclose(c, cov, atol=0.12 * np.sqrt(np.outer(np.diag(cov), np.diag(cov))))
    assert 2 <= np.mean(depths) < md


@pytest.mark.parametrize("target", ["gaussian", "model"])
def test_one_level_tree_is_a_metropolis_leapfrog_step(target):
    """With max_depth = 1 the tree is the start point and one leapfrog step in
    the drawn direction, and joining it is a Metropolis move with probability
    min(1, exp(H0 - H1)) (Hoffman & Gelman 2014; Neal 2011, Sec. 5.3)."""
    if target == "gaussian":
        pg = _gaussian(np.diag([1.0, 2.0, 0.5]))
        q0 = np.array([0.3, -1.0, 0.2])
        minv = np.array([1.0, 0.5, 2.0])
        eps = 0.4
        split = None
    else:
        w, m, nu_t, nu_e, counts = mock_case("c0fd")
        ch = w.chains[0]
        tying = w.free
        mu = np.full(len(tying), fi.PRIOR_MU_ALPHA)
        sig = np.full(len(tying), fi.PRIOR_SIGMA_ALPHA)
        u0 = np.log(np.array([ch.bias[r[0], c] for r, c in tying]))
        nv = nu_t.size
        split = nv

        def pg(q):
            pot, gnu, gu = hmc.potential_and_grad(m, q[:nv].reshape(nu_t.shape), q[nv:], ch.bias, tying,
                                                  mu, sig, counts)
            return pot, np.concatenate([gnu.ravel(), gu])
        q0 = np.concatenate([nu_t.ravel(), u0])
        minv = np.concatenate([np.ones(nv), np.full(len(u0), 1e-3)])
        eps = 0.02
    rng = np.random.default_rng(3)
    z = rng.standard_normal(q0.size)
    p0 = z / np.sqrt(minv)
    for direction in (0.2, 0.7):
        v = 1 if direction >= 0.5 else -1
        if split is None:
            g = lambda q, u: (*pg(q)[:2], np.zeros(1))
            q1, _, _, _, h0, h1 = hmc.leapfrog(g, q0, np.zeros(1), p0, np.zeros(1), minv, 1.0, v * eps, 1)
        else:
            g = lambda q, u: (lambda r: (r[0], r[1][:split], r[1][split:]))(pg(np.concatenate([q, u])))
            qn, qu, _, _, h0, h1 = hmc.leapfrog(g, q0[:split], q0[split:], p0[:split], p0[split:],
                                                minv[:split], minv[split:], v * eps, 1)
            q1 = np.concatenate([qn, qu])
        paccept = min(1.0, math.exp(h0 - h1))
        for join in (0.5 * paccept, min(0.999, paccept + 0.5 * (1 - paccept)) if paccept < 1 else None):
            if join is None:
                continue
            uni = np.array([direction, join, 0.3])
            t = nuts.transition(pg, q0, z, minv, eps, uni, 1)
            assert t.n_leapfrog == 1 and t.h0 == pytest.approx(h0, rel=1e-12)
            assert t.accept_stat == pytest.approx(paccept, rel=1e-9)
            want = q1 if join < paccept else q0
            assert np.allclose(t.q, want, rtol=1e-12, atol=1e-12)
            assert t.depth == 1


def _recursive_stop(ps, minv):
    """Stopping leaf of a subtree whose leaves' momenta are `ps` (creation
    order), by the recursive BuildTree of Hoffman & Gelman 2014 with the
    generalised criterion: a subtree is built as two halves, the right half
    only if the left one did not turn, and the whole is checked last.  Returns
    the number of leaves made before stopping, and whether it turned."""
    def build(lo, size):
        if size == 1:
            return 1, False
        n1, t1 = build(lo, size // 2)
        if t1:
            return n1, True
        n2, t2 = build(lo + size // 2, size // 2)
        if t2:
            return n1 + n2, True
        blk = ps[lo:lo + size]
        rho = np.sum(blk, axis=0)
        turn = float(np.dot(minv * blk[0], rho)) <= 0 or float(np.dot(minv * blk[-1], rho)) <= 0
        return n1 + n2, turn
    return build(0, len(ps))


def test_stopping_rule_matches_the_recursive_tree():
    """On 2-D oscillators with unequal frequencies, the leaves made and the
    depth reached agree with an explicit trajectory checked by the recursive
    formulation of the tree (all directions drawn to the right), over step
    sizes where the trajectory ends by a turn inside a new subtree and where it
    ends by a turn of the whole tree."""
    md = 8
    uni = np.full(nuts.n_uniforms(md), 0.9)
    reasons = set()
    for scale in (0.3, 0.05, 1.0):
        pg = _gaussian(np.diag([1.0, scale]))
        q0 = np.array([0.5, -0.2])
        z = np.array([0.9, 0.4])
        for eps in (0.03, 0.05, 0.08, 0.13, 0.2, 0.31, 0.45, 0.7):
            t = nuts.transition(pg, q0, z, 1.0, eps, uni, md)
            # explicit trajectory to the right, 2^md - 1 leaves
            q, p = q0.copy(), z.copy()
            u, g = pg(q)
            leaves = []
            for _ in range((1 << md) - 1):
                p = p - 0.5 * eps * g
                q = q + eps * p
                u, g = pg(q)
                p = p - 0.5 * eps * g
                leaves.append(p)
            n_made, depth, reason = 0, 0, "depth"
            rho = z.copy()
            for j in range(md):
                sub = leaves[(1 << j) - 1:(1 << (j + 1)) - 1]
                nm, turned = _recursive_stop(sub, 1.0)
                n_made += nm
                if turned:
                    reason = "subtree"
                    break
                depth = j + 1
                rho = rho + np.sum(sub, axis=0)
                if float(np.dot(z, rho)) <= 0 or float(np.dot(sub[-1], rho)) <= 0:
                    reason = "tree"
                    break
            assert (t.n_leapfrog, t.depth) == (n_made, depth), (scale, eps)
            reasons.add(reason)
    assert {"subtree", "tree"} <= reasons


def test_divergence_ends_the_tree():
    """A potential whose energy blows up past 1000 stops the trajectory."""
    pg = lambda q: (float(np.sum(q ** 6)), 6 * q ** 5)
    t = nuts.transition(pg, np.array([1.5, 1.5]), np.array([3.0, 3.0]), 1.0, 0.5,
                        np.full(nuts.n_uniforms(5), 0.9), 5)
    assert t.diverging and t.depth < 5


def test_dual_averaging_converges_to_the_target_acceptance():
    """With a deterministic acceptance a(eps) = exp(-eps), the averaged step
    tends to the root of a(eps) = 0.8."""
    da = nuts.DualAveraging(1.0)
    eps = 1.0
    for _ in range(3000):
        eps = da.update(math.exp(-eps))
    assert da.final() == pytest.approx(-math.log(0.8), rel=0.02)


def test_welford_matches_numpy_variance():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((500, 7)) * np.arange(1, 8) + 3.0
    w = nuts.Welford(7)
    for row in x:
        w.add(row)
    assert np.allclose(w.mean, x.mean(0), rtol=1e-12)
    assert np.allclose(w.variance(), x.var(0, ddof=1), rtol=1e-10)


def test_window_schedule_of_a_thousand_warmup_iterations():
    """Stan's documented default: after a 75-iteration buffer, windows of 25,
    50, 100, 200 and 500 iterations, then a 50-iteration terminal buffer."""
    assert nuts.window_ends(1000) == [100, 150, 250, 450, 950]
    assert nuts.window_ends(100) == []


@pytest.mark.parametrize("scheme", ["blanes2", "yoshida4"])
def test_samples_keep_a_gaussian_invariant_with_other_schemes(scheme):
    """Leaves made with the two-stage or the fourth-order step: a 2-D
    Gaussian's moments within a few Monte Carlo errors."""
    cov = np.array([[1.0, 0.5], [0.5, 2.0]])
    pg = _gaussian(cov)
    rng = np.random.default_rng(21)
    q = np.zeros(2)
    draws = []
    md = 5
    for it in range(3000):
        t = nuts.transition(pg, q, rng.standard_normal(2), 1.0, 0.4,
                            rng.uniform(size=nuts.n_uniforms(md)), md, scheme=scheme)
        q = t.q
        draws.append(q)
    x = np.array(draws[300:])
    assert np.all(np.abs(x.mean(0)) < 0.15)
    assert np.allclose(np.cov(x.T), cov, atol=0.15 * np.sqrt(np.outer(np.diag(cov), np.diag(cov))))
