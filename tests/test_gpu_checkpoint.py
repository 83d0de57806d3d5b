"""Displacement-field checkpointing (FZW_PLAN_CHECKPOINT): a plan that keeps no
first-order Hessian between the forward model and the adjoint (recomputed from
nu in the adjoint) gives the log-likelihood and both gradients of a plan that
keeps it, bit for bit: on meshes whose LPT step is fused with its z transforms
(64^3, 128^3) and on the one that is not (96^3, radial RSD), in a
graph-captured trajectory of a batch of two meshes, and for the bispectrum,
whose scratch fields move to the tensor buffers.  Its workspace is smaller by
at least the six Hessian fields per chain; against the oracle it follows the
rule of tests/helpers.py."""
import dataclasses

import numpy as np
import pytest

import fzw_inputs as fi
from tests.helpers import GRAD_TOL, LOGL_TOL, Floor, fp32, mock_case

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)

from tests.gpu_helpers import dev, dev_counts, host, plan_for, relnorm  # noqa: E402

RADIAL = 3


@pytest.mark.parametrize("case", [("c2", 64, -1), ("c2", 96, RADIAL), ("c1", None, -1)],
                         ids=["c2-64", "c2-96-radial", "c1-128"])
def test_checkpointed_plan_equals_the_stored_one(case):
    from paper_2506_03969_amd import FIELD_DPSI, FIELD_DRHO, FzwError
    name, n, rsd = case
    w, m, nu_t, nu_e, counts = mock_case(name, n, rsd_axis=None if rsd < 0 else rsd)
    ch = w.chains[0]
    nu = fp32(fi.near_truth_noise(ch))
    b = fp32(ch.bias)
    plans = [plan_for(w), plan_for(w, checkpoint=True)]
    res, fwd, fields = [], [], []
    for p in plans:
        p.set_counts(0, dev_counts(counts))
        res.append([t.clone() for t in p.value_and_grad(dev(nu.ravel()), dev(b[None]))])
        fields.append([p.get_field(0, k).clone() for k in (4, 5, FIELD_DRHO, FIELD_DPSI, FIELD_DPSI + 2)])
        fwd.append(p.forward(dev(nu.ravel()), dev(b[None])).clone())
    ws = [p.workspace_bytes for p in plans]
    print(name, n, "workspace %.1f MB stored, %.1f MB checkpointed" % (ws[0] / 1e6, ws[1] / 1e6))
    assert ws[1] <= ws[0] - 6 * ch.n ** 3 * 4
    for a, c in zip(res[0], res[1]):
        assert torch.equal(a, c)
    for a, c in zip(fields[0], fields[1]):
        assert torch.equal(a, c)
    assert torch.equal(fwd[0], fwd[1])
    with pytest.raises(FzwError, match="status -5"):
        plans[1].get_field(0, 0)                 # delta_L is the trace of the stored phi
    # the checkpointed plan against the oracle
    logl, dnu, dbias = res[1]
    ref_l, ref_dnu, ref_db = m.value_and_grad(nu, b, counts)
    e_l = abs(float(host(logl)[0]) - ref_l) / abs(ref_l)
    e_nu = relnorm(host(dnu).reshape(nu.shape), ref_dnu)
    e_bn = relnorm(host(dbias).reshape(b.shape), ref_db)
    fl = Floor(m, nu, b, counts, ref_dnu, ref_db)
    ok_nu = fl.holds_nu(e_nu)
    print(name, n, "checkpointed vs oracle: logL %.2e dnu %.2e dbias %.2e (floor %d draws: %.2e)" % (
        e_l, e_nu, e_bn, fl.draws, fl.nu_f))
    assert e_l < LOGL_TOL and e_bn < GRAD_TOL and ok_nu
    if n == 64:
        # the bispectrum's scratch fields (the tensor buffers of a checkpointed plan)
        delta = dev(fi.white_noise(ch, fi.ROLE_MISC).ravel())
        kf = 2 * np.pi / ch.box
        th = [0.4, 1.5, 2.6]
        bs = [host(p.bispectrum(delta, 0.1, 0.2, 2 * kf, th, mesh_n=ch.n)) for p in plans]
        assert np.array_equal(bs[0], bs[1])


def test_checkpointed_trajectory_equals_the_stored_one():
    """A graph-captured leapfrog trajectory of a batch of a 32^3 and a 16^3
    chain (two mesh groups on their own streams): the same end state and
    Hamiltonians, bit for bit."""
    w = fi.workload("c3")
    chains = [fi.Chain(32, 128.0, w.chains[0].bias, 1.0, w.chains[0].seed_key),
              fi.Chain(16, 64.0, w.chains[12].bias, 1.0, w.chains[12].seed_key)]
    ww = dataclasses.replace(w, chains=chains)
    mu, sig = fi.prior_arrays(ww)
    rng = np.random.default_rng(5)
    cnts = [rng.poisson(1.0, size=(c.n,) * 3).astype(np.uint16) for c in chains]
    nu0 = np.concatenate([fi.white_noise(c, fi.ROLE_EVAL_NU).astype(np.float32).ravel() for c in chains])
    pn0 = rng.standard_normal(nu0.size).astype(np.float32)
    u0 = np.stack([fi.free_start(ww, c) for c in chains]).astype(np.float32)
    pu0 = rng.standard_normal(u0.shape).astype(np.float32)
    out = []
    for ck in (False, True):
        p = plan_for(ww, checkpoint=ck)
        p.set_sampling(fi.tie_array(ww), mu, sig)
        for i, c in enumerate(cnts):
            p.set_counts(i, dev_counts(c))
        nu, pn, u, pu = dev(nu0), dev(pn0), dev(u0), dev(pu0)
        base = dev(np.stack([c.bias for c in chains]))
        h0, h1 = p.leapfrog(nu, u, pn, pu, base, torch.ones_like(nu), torch.full_like(u, 1e-2),
                            dev(np.full(2, 1e-3)), 3)
        out.append([t.clone() for t in (nu, u, pn, pu, h0, h1)])
    print("H0", host(out[0][4]), "H1", host(out[0][5]))
    for a, c in zip(out[0], out[1]):
        assert torch.equal(a, c)
