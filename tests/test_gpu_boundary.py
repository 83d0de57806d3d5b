"""The C-ABI boundary beyond the model's numbers: the torch.autograd front door,
which intermediate fields a call leaves, and non-finite states.

Non-finite states are forced from the host (NaN or huge white noise handed to
the library); every kernel still runs to completion on them: the deposit
replaces a displacement that is not finite (or reaches 2^30 cells) by zero, so
no index or weight is undefined, and flags the chain.
"""
import numpy as np
import pytest

import fzw_inputs as fi
from tests.helpers import mock_case

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)

from tests.gpu_helpers import dev, dev_counts, host, plan_for, relnorm  # noqa: E402


def _two_chain_plan(n=16):
    """Two chains of the 16^3 workload (same mesh: one batched group), each
    with its own mock data."""
    import dataclasses
    w, m, nu_t, nu_e, counts = mock_case("c0fd")
    ch = w.chains[0]
    ch2 = fi.Chain(ch.n, ch.box, ch.bias * np.array([1.05, 1.0, 1.0, 1.0]), ch.mean_count, (ch.seed_key[0], 1))
    ww = dataclasses.replace(w, chains=[ch, ch2])
    p = plan_for(ww)
    for c in range(2):
        p.set_counts(c, dev_counts(counts))
    # two well-conditioned states of the mock: near the data's noise, and the noise itself
    nus = [fi.near_truth_noise(ch).astype(np.float32), nu_t.astype(np.float32)]
    bias = np.stack([ch.bias, ch2.bias]).astype(np.float32)
    return ww, m, p, nus, [counts, counts], bias


@pytest.mark.parametrize("shape", ["flat", "4d"])
def test_loglikelihood_autograd_function(shape):
    """LogLikelihood.apply(nu, b, plan) is logL per chain, and backward of a
    weighted sum gives w_c times chain c's gradient (against value_and_grad
    and against the oracle on the same float32 inputs)."""
    from paper_2506_03969_amd import LogLikelihood
    ww, m, p, nus, cnts, bias = _two_chain_plan()
    n = ww.chains[0].n
    flat = np.concatenate([x.ravel() for x in nus])
    nu = dev(flat if shape == "flat" else flat.reshape(2, n, n, n)).requires_grad_(True)
    b = dev(bias).requires_grad_(True)
    logl = LogLikelihood.apply(nu, b, p)
    assert logl.shape == (2,) and logl.dtype == torch.float64
    wgt = torch.tensor([0.7, -1.9], dtype=torch.float64, device="cuda")
    (wgt * logl).sum().backward()
    l2, g2, b2 = p.value_and_grad(nu.detach().contiguous(), b.detach().contiguous())
    assert torch.equal(logl.detach(), l2)
    gn = nu.grad.reshape(2, -1)
    gr = g2.reshape(2, -1)
    for c in range(2):
        assert torch.equal(gn[c], gr[c] * wgt[c].float())
        assert torch.equal(b.grad[c], b2[c] * wgt[c].float())
    # and chain by chain against the oracle
    for c in range(2):
        ch = ww.chains[c]
        ref_l, ref_g, ref_b = m.value_and_grad(nus[c].astype(np.float64), bias[c].astype(np.float64), cnts[c])
        assert abs(float(logl[c]) - ref_l) < 1e-4 * abs(ref_l)
        got = host(gn[c]).reshape(ref_g.shape) / float(wgt[c])
        assert relnorm(got, ref_g) < 1e-4


def test_get_field_reports_what_the_last_call_left():
    """After a gradient evaluation the displacement and tensor buffers hold
    cotangents: those fields are refused, the density, log f (and delta_L on
    the fused meshes) still match the forward model's, and the cotangents of
    rho and Psi are available; after a forward call it is the other way
    round."""
    from paper_2506_03969_amd import FIELD_DPSI, FIELD_DRHO, FzwError
    w, m, nu_t, nu_e, counts = mock_case("c2", 32)
    p = plan_for(w)
    with pytest.raises(FzwError, match="status -5"):
        p.get_field(0, 4)                     # nothing evaluated yet
    p.set_counts(0, dev_counts(counts))
    nu = dev(fi.near_truth_noise(w.chains[0]).ravel())
    bias = dev(w.chains[0].bias[None])
    p.forward(nu, bias)
    fwd = {k: p.get_field(0, k).clone() for k in (0, 1, 4, 5, 6, 17)}
    for k in (FIELD_DRHO, FIELD_DPSI):
        with pytest.raises(FzwError, match="status -5"):
            p.get_field(0, k)
    p.value_and_grad(nu, bias)
    for k in (1, 2, 3, 6, 11, 12, 17):
        with pytest.raises(FzwError, match="status -5"):
            p.get_field(0, k)
    for k in (0, 4, 5):
        assert torch.equal(p.get_field(0, k), fwd[k])
    drho = p.get_field(0, FIELD_DRHO)
    dpsi = [p.get_field(0, FIELD_DPSI + j) for j in range(3)]
    assert bool(torch.isfinite(drho).all()) and float(drho.abs().max()) > 0
    assert all(bool(torch.isfinite(d).all()) for d in dpsi)
    with pytest.raises(FzwError, match="status -1"):
        p.get_field(0, 22)
    p.forward(nu, bias)
    assert torch.equal(p.get_field(0, 1), fwd[1])


def _finite_reference(p, nu, bias):
    l, g, b = p.value_and_grad(nu, bias)
    return l.clone(), g.clone(), b.clone()


@pytest.mark.parametrize("poison", ["nan", "huge"])
def test_nonfinite_state_is_flagged_and_the_plan_stays_usable(poison):
    """White noise with a NaN (or of size 1e30, whose displacements overflow)
    gives logL = NaN and the chain's flags, the other chain of the batch is
    untouched, and the next call on the same plan reproduces the earlier
    finite result bit for bit."""
    from paper_2506_03969_amd import NF_LOGL, NF_STATE
    ww, m, p, nus, cnts, bias = _two_chain_plan()
    nu = dev(np.concatenate([x.ravel() for x in nus]))
    b = dev(bias)
    l0, g0, b0 = _finite_reference(p, nu, b)
    ok, flags = p.check_finite()
    assert ok and flags == [0, 0]
    bad = nu.clone()
    n3 = ww.chains[0].n ** 3
    if poison == "nan":
        bad[n3 + 123] = float("nan")
    else:
        bad[n3:] = 1e30 * nu[n3:]        # (a constant would have no k != 0 modes)
    lf = p.forward(bad, b)
    ok, flags = p.check_finite()
    print(poison, "logL", host(lf), "flags", flags)
    assert not ok
    assert flags[0] == 0
    assert flags[1] & NF_LOGL and flags[1] & NF_STATE
    assert float(lf[0]) == float(l0[0]) and np.isnan(float(lf[1]))
    l1, g1, b1 = p.value_and_grad(bad, b)
    ok, flags = p.check_finite()
    assert not ok and flags[0] == 0 and flags[1] & NF_LOGL
    dev_flags = p.nonfinite_flags()
    assert host(dev_flags).astype(int).tolist() == flags
    assert float(l1[0]) == float(l0[0]) and np.isnan(float(l1[1]))
    assert torch.equal(g1[:n3], g0[:n3]) and torch.equal(b1[0], b0[0])
    # the plan is still usable: the finite state again, bit for bit
    l2, g2, b2 = p.value_and_grad(nu, b)
    ok, flags = p.check_finite()
    assert ok and flags == [0, 0]
    assert torch.equal(l2, l0) and torch.equal(g2, g0) and torch.equal(b2, b0)


def test_nonfinite_trajectory_has_nonfinite_hamiltonian():
    """A leapfrog trajectory started from a NaN state ends with a non-finite
    H (the Metropolis step rejects it) and the Hamiltonian flag; the next
    trajectory from a finite state on the same plan is finite and unflagged."""
    from paper_2506_03969_amd import NF_HAMILTONIAN
    ww, m, p, nus, cnts, bias = _two_chain_plan()
    mu, sig = fi.prior_arrays(ww)
    p.set_sampling(fi.tie_array(ww), mu, sig)
    nu = dev(np.concatenate([x.ravel() for x in nus]))
    u = dev(np.stack([fi.free_start(ww, ch) for ch in ww.chains]))
    base = dev(bias)
    rng = np.random.default_rng(2)
    pn0 = rng.standard_normal(nu.numel()).astype(np.float32)
    pu0 = rng.standard_normal(tuple(u.shape)).astype(np.float32)
    minv = torch.ones_like(nu)
    minv_u = torch.full_like(u, 1e-2)
    step = dev(np.full(2, 1e-3))

    def run(x):
        q, uu, pn, pu = x.clone(), u.clone(), dev(pn0), dev(pu0)
        h0, h1 = p.leapfrog(q, uu, pn, pu, base, minv, minv_u, step, 2)
        return host(h0), host(h1)

    bad = nu.clone()
    bad[7] = float("nan")
    h0, h1 = run(bad)
    ok, flags = p.check_finite()
    print("NaN start: H0", h0, "H1", h1, "flags", flags)
    assert not np.isfinite(h1[0]) and not np.isfinite(h0[0])
    assert flags[0] & NF_HAMILTONIAN and not ok
    assert np.all(np.isfinite(h1[1:])) and flags[1] == 0
    h0, h1 = run(nu)
    ok, flags = p.check_finite()
    assert ok and np.all(np.isfinite(h0)) and np.all(np.isfinite(h1))


def test_tracer_in_an_empty_cell_matches_the_oracle():
    """A tracer placed in a cell that no particle reaches (rho = 0, so x is the
    floor 1e-6): the likelihood is finite and very negative, evaluated in
    log space on both sides, and matches the oracle on the same float32
    inputs; the gradient is finite (zero derivative below the floor)."""
    w, m, nu_t, nu_e, counts = mock_case("c2", 32)
    ch = w.chains[0]
    nu = nu_e.astype(np.float32).astype(np.float64)
    bias = ch.bias.astype(np.float32).astype(np.float64)
    st = m.forward(nu, bias)
    empty = np.flatnonzero(st["rho"].ravel() == 0.0)
    if empty.size == 0:
        pytest.skip("no empty cell in this state")
    c = counts.copy().reshape(-1)
    c[empty[: min(3, empty.size)]] += 2
    c = c.reshape(counts.shape)
    p = plan_for(w)
    p.set_counts(0, dev_counts(c))
    logl, dnu, dbias = p.value_and_grad(dev(nu.ravel()), dev(bias[None]))
    ok, flags = p.check_finite()
    ref_l, ref_g, ref_b = m.value_and_grad(nu, bias, c)
    print("empty cells %d, logL gpu %.9e oracle %.9e" % (empty.size, float(logl[0]), ref_l))
    assert ok and np.isfinite(ref_l) and ref_l < -1e4
    assert abs(float(logl[0]) - ref_l) < 1e-4 * abs(ref_l)
    assert bool(torch.isfinite(dnu).all()) and bool(torch.isfinite(dbias).all())
