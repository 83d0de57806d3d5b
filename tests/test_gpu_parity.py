"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

Both sides get the same float32 inputs; tolerances and the conditioning
floor follow the rule in tests/helpers.py: fields 1e-5 normwise,
log-likelihood 1e-4 relative, gradients and cotangents 1e-4 normwise,
bias-table entries 1e-4 relative to max(|g|, 1e-3 max|g|), or ten times the
oracle's own movement under a 5e-7 relative perturbation of its input where
that is larger.
"""
import numpy as np
import pytest

import fzw_inputs as fi
from tests.helpers import (FIELD_TOL, GRAD_TOL, LOGL_TOL, Floor, conditioned_counts, fp32, mock_case,
                           off_face, oracle_gradient)

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)

from tests.gpu_helpers import bias_entry_error, dev, dev_counts, host, plan_for, relnorm  # noqa: E402

CASES = [("c0fd", None), ("c0", None), ("c2", 32), ("c2", 64), ("c1", None)]


def _ids(c):
    return "%s-%s" % c


@pytest.fixture(scope="module")
def fft_plans():
    w = fi.workload("c0")
    plans = {}
    for n in (16, 32, 64, 96, 128, 256):
        ww = fi.small_variant(w, n)
        plans[n] = plan_for(ww)
    return plans


@pytest.mark.parametrize("n", [16, 32, 64, 96, 128, 256])
def test_fft_matches_numpy(fft_plans, n):
    p = fft_plans[n]
    rng = np.random.default_rng(n)
    x = rng.standard_normal((2, n, n, n)).astype(np.float32)
    got = p.fft_r2c(dev(x)).cpu().numpy()
    ref = np.fft.rfftn(x.astype(np.float64), axes=(1, 2, 3))
    err = relnorm(got, ref)
    print("fft r2c n=%d err=%.2e" % (n, err))
    assert err < 2e-6
    back = host(p.fft_c2r(torch.from_numpy(ref.astype(np.complex64)).cuda()))
    err2 = relnorm(back, x.astype(np.float64) * n ** 3)
    print("fft c2r n=%d err=%.2e" % (n, err2))
    assert err2 < 2e-6


def _state(name, n, which, tau_sc=None, rsd=None):
    """Workload, oracle, white noise of the state and counts; the noise is
    the float32 rounding the GPU is handed (as float64, for the oracle)."""
    w, m, nu_t, nu_e, counts = mock_case(name, n, tau_sc, rsd_axis=rsd)
    if which == "truth":
        nu = nu_t
    elif which == "near":
        nu = fi.near_truth_noise(w.chains[0])
    else:
        nu = nu_e
    return w, m, fp32(nu), counts


def _gpu_forward(name, n, which="truth", tau_sc=None, rsd=None):
    """Plan with the counts set; returns the state and the bias table as the
    float32 values both sides use (the table also as a device tensor)."""
    w, m, nu, counts = _state(name, n, which, tau_sc, rsd)
    ch = w.chains[0]
    p = plan_for(w)
    p.set_counts(0, dev_counts(counts))
    b = fp32(ch.bias)
    return w, m, nu, counts, p, dev(b.reshape(1, -1, 4)), b


RADIAL = 3   # radial RSD about the box centre
RADIAL_CASES = [("c0fd", None), ("c2", 32), ("c2", 64), ("c2", 96)]


@pytest.mark.parametrize("case,rsd", [(c, None) for c in CASES] + [(c, RADIAL) for c in RADIAL_CASES],
                         ids=lambda x: _ids(x) if isinstance(x, tuple) else ("radial" if x == RADIAL else "los"))
@pytest.mark.parametrize("which", ["truth", "near", "eval"])
def test_forward_stages_and_logl(case, rsd, which):
    name, n = case
    w, m, nu, counts, p, bias, b = _gpu_forward(name, n, which, rsd=rsd)
    logl, nbar = p.forward(dev(nu.ravel()), bias, want_nbar=True)
    st = m.forward(nu, b, counts)
    errs = {
        "delta_L": relnorm(host(p.get_field(0, 0)), st["dl"]),
        "psi": relnorm(np.stack([host(p.get_field(0, k)) for k in (1, 2, 3)]), st["psi"]),
        "rho": relnorm(host(p.get_field(0, 4)), st["rho"]),
        # f = exp(log f): log f itself is ill-conditioned in near-empty cells,
        # where it is ~ -(rho_th / x) and inherits the relative error of x
        "f": relnorm(np.exp(host(p.get_field(0, 5)).ravel()), st["f"]),
        "nbar": relnorm(host(nbar), st["nbar"]),
    }
    for wi in range(len(w.web.kinds)):
        t_gpu = np.stack([host(p.get_field(0, 6 + 6 * wi + k)) for k in range(6)])
        errs["T%d" % wi] = relnorm(t_gpu, np.stack(st["tens"][wi]))
    lg = float(host(logl)[0])
    errs["logL"] = abs(lg - st["logl"]) / abs(st["logl"])
    print(name, n, which, " ".join("%s=%.2e" % kv for kv in errs.items()))
    for k, v in errs.items():
        tol = LOGL_TOL if k == "logL" else FIELD_TOL
        assert v < tol, (k, v)


GRAD_CASES = ([(c, "truth", None, None) for c in CASES] + [(c, "near", None, None) for c in CASES]
              + [(c, "truth", 0.0, None) for c in CASES[1:]] + [(c, "eval", None, None) for c in CASES[1:]]
              + [(c, which, None, RADIAL) for c in RADIAL_CASES for which in ("truth", "near")])


def _gid(x):
    (name, n), which, tau, rsd = x
    return "%s-%s-%s%s%s" % (name, n, which, "-exact_hinge" if tau == 0.0 else "",
                             "-radial" if rsd == RADIAL else "")


@pytest.mark.parametrize("gcase", GRAD_CASES, ids=_gid)
def test_gradient(gcase):
    """The mock data as drawn.  logL within 1e-4 and the bias-table gradient
    within 1e-4 normwise at every state; d logL/d nu and the bias entries
    within 1e-4 or ten times the oracle's conditioning floor.  The floor
    exceeds 1e-4 with the exact spherical-collapse hinge (its derivative
    diverges at delta_L = 3/2), where a particle sits within float32 noise of
    a cell face, and for bias entries at the data's own parameters (their
    voxel sums cancel to ~1%).  At the independently drawn state ('eval')
    tracers sit in cells at the density floor, where a cell crossing it under
    float32 rounding changes d logL/d nu by up to tens of times its norm: that
    state's d/dnu is compared on the conditioned data of
    test_gradient_conditioned instead."""
    (name, n), which, tau, rsd = gcase
    w, m, nu, counts, p, bias, b = _gpu_forward(name, n, which, tau, rsd)
    logl, dnu, dbias = p.value_and_grad(dev(nu.ravel()), bias)
    ref_l, ref_dnu, ref_db, st = oracle_gradient(m, nu, b, counts)
    e_l = abs(float(host(logl)[0]) - ref_l) / abs(ref_l)
    g = host(dnu).reshape(nu.shape)
    gb = host(dbias).reshape(ref_db.shape)
    e_nu = relnorm(g, ref_dnu)
    e_bn = relnorm(gb, ref_db)
    e_b = bias_entry_error(gb, ref_db)
    fl = Floor(m, nu, b, counts, ref_dnu, ref_db, st["dbias_abs"])
    ok_nu = which == "eval" or fl.holds_nu(e_nu)
    ok_b = fl.holds_bias(gb)
    print(_gid(gcase), "logL=%.2e dnu=%.2e dbias norm=%.2e entry=%.2e (floor %d draws: nu %.2e bias %.2e)" % (
        e_l, e_nu, e_bn, e_b, fl.draws, fl.nu_f, fl.bias_f))
    assert e_l < LOGL_TOL
    assert np.all(np.isfinite(g)) and np.all(np.isfinite(gb))
    assert e_bn < GRAD_TOL
    assert ok_nu and ok_b


COND_CASES = ([(c, which, None, None) for c in CASES for which in ("near", "eval")]
              + [(c, "truth", 0.0, None) for c in (("c2", 64), ("c1", None))]
              + [(("c2", 64), "eval", None, RADIAL)])


@pytest.mark.parametrize("gcase", COND_CASES, ids=_gid)
def test_gradient_conditioned(gcase):
    """Conditioned data (the mock counts without tracers in cells whose
    density at the state is below 0.05 of the mean, so that every per-voxel
    term is bounded), the eval state included.  The adjoint's intermediate
    cotangents are compared element by element with the oracle's at the fixed
    1e-4, no floor: d logL/d rho over every voxel, d logL/d Psi over the
    particles more than 1e-5 cells from every cell face.  d logL/d nu and the
    bias entries within 1e-4 or ten times the floor (a face crossing, the
    exact hinge), the bias gradient within 1e-4 normwise."""
    from paper_2506_03969_amd import FIELD_DPSI, FIELD_DRHO
    (name, n), which, tau, rsd = gcase
    w, m, nu, counts, p, bias, b = _gpu_forward(name, n, which, tau, rsd)
    cc = conditioned_counts(m, nu, b, counts)
    p.set_counts(0, dev_counts(cc))
    logl, dnu, dbias = p.value_and_grad(dev(nu.ravel()), bias)
    drho = host(p.get_field(0, FIELD_DRHO))
    dpsi = np.stack([host(p.get_field(0, FIELD_DPSI + j)) for j in range(3)])
    st = m.forward(nu, b, cc)
    ref_dnu, ref_db = m.adjoint(st)
    keep = off_face(st["pos"])
    e = {"logL": abs(float(host(logl)[0]) - st["logl"]) / abs(st["logl"]),
         "drho": relnorm(drho, st["drho"]),
         "dpsi_off_face": relnorm(dpsi.reshape(3, -1)[:, keep], st["dpsi"].reshape(3, -1)[:, keep]),
         "dpsi": relnorm(dpsi, st["dpsi"]),
         "dnu": relnorm(host(dnu).reshape(nu.shape), ref_dnu),
         "dbias": relnorm(host(dbias).reshape(ref_db.shape), ref_db),
         "dbias_entry": bias_entry_error(host(dbias).reshape(ref_db.shape), ref_db)}
    fl = Floor(m, nu, b, cc, ref_dnu, ref_db, st["dbias_abs"])
    ok_nu, ok_b = fl.holds_nu(e["dnu"]), fl.holds_bias(host(dbias).reshape(ref_db.shape))
    print(_gid(gcase), "tracers removed %d, particles near a face %d:" % (
        int(np.sum(counts) - np.sum(cc)), int((~keep).sum())),
        " ".join("%s=%.2e" % kv for kv in e.items()), "(floor %d draws: nu %.2e bias %.2e)" % (
        fl.draws, fl.nu_f, fl.bias_f))
    assert e["logL"] < LOGL_TOL
    assert e["drho"] < GRAD_TOL and e["dpsi_off_face"] < GRAD_TOL
    assert e["dbias"] < GRAD_TOL
    assert ok_nu and ok_b


def test_likelihood_count_range():
    """Counts across every branch of the likelihood pass against the oracle:
    0 and 1, 2..9 and 10..64 (the two queues of its float64 sum, with
    partial batches left for the end) and above 64 (the float64 special
    functions).  One voxel in ten gets 8..59 more tracers, one in a hundred
    65..399 more."""
    w, m, nu, counts, p, bias, b = _gpu_forward("c2", 32, "truth")
    rng = np.random.default_rng(77)
    c = counts.astype(np.int64).reshape(-1).copy()
    idx = rng.permutation(c.size)
    k = c.size // 10
    c[idx[:k]] += rng.integers(8, 60, k)
    c[idx[k:k + k // 10]] += rng.integers(65, 400, k // 10)
    c = c.reshape(counts.shape)
    print("counts: n<=1 %d, 2..9 %d, 10..64 %d, >64 %d" % (
        np.sum(c <= 1), np.sum((c >= 2) & (c <= 9)), np.sum((c >= 10) & (c <= 64)), np.sum(c > 64)))
    assert np.sum(c > 64) > 0 and np.sum((c >= 10) & (c <= 64)) > 0
    p.set_counts(0, dev_counts(c))
    logl, dnu, dbias = p.value_and_grad(dev(nu.ravel()), bias)
    lf = p.forward(dev(nu.ravel()), bias)
    ref_l, ref_dnu, ref_db, st = oracle_gradient(m, nu, b, c)
    e_l = abs(float(host(logl)[0]) - ref_l) / abs(ref_l)
    g = host(dnu).reshape(nu.shape)
    gb = host(dbias).reshape(ref_db.shape)
    e_nu, e_bn, e_b = relnorm(g, ref_dnu), relnorm(gb, ref_db), bias_entry_error(gb, ref_db)
    fl = Floor(m, nu, b, c, ref_dnu, ref_db, st["dbias_abs"])
    ok_nu, ok_b = fl.holds_nu(e_nu), fl.holds_bias(gb)
    print("count range: logL=%.2e dnu=%.2e dbias=%.2e entry %.2e (floor %d draws: nu %.2e bias %.2e)" % (
        e_l, e_nu, e_bn, e_b, fl.draws, fl.nu_f, fl.bias_f))
    assert float(host(lf)[0]) == float(host(logl)[0])
    assert e_l < LOGL_TOL
    assert e_bn < GRAD_TOL and ok_nu and ok_b


def test_bitwise_determinism():
    w, m, nu, counts, p, bias, b = _gpu_forward("c2", 32, "eval")
    x = dev(nu.ravel())
    a = [t.clone() for t in p.value_and_grad(x, bias)]
    b = [t.clone() for t in p.value_and_grad(x, bias)]
    for u, v in zip(a, b):
        assert torch.equal(u, v)


def test_batched_chains_equal_single_chain_results():
    """Chains of equal mesh share launches; each chain's result equals the one
    from a plan holding that chain alone, bit for bit."""
    w = fi.workload("c3")
    sel = [0, 1, 12]          # two 64^3 chains and one 96^3 chain
    chains = [w.chains[i] for i in sel]
    small = [fi.Chain(32, 128.0, c.bias, 1.0, c.seed_key) for c in chains[:2]] + [
        fi.Chain(16, 64.0, chains[2].bias, 1.0, chains[2].seed_key)]
    import dataclasses
    ww = dataclasses.replace(w, chains=small)
    rng = np.random.default_rng(0)
    nus = [fi.white_noise(c, fi.ROLE_EVAL_NU).astype(np.float32) for c in small]
    cnts = [rng.poisson(1.0, size=(c.n,) * 3).astype(np.uint16) for c in small]
    pb = plan_for(ww)
    for i, c in enumerate(cnts):
        pb.set_counts(i, dev_counts(c))
    nu_all = dev(np.concatenate([x.ravel() for x in nus]))
    bias_all = dev(np.stack([c.bias for c in small]))
    lb, gb, bb = pb.value_and_grad(nu_all, bias_all)
    for i, c in enumerate(small):
        ps = plan_for(dataclasses.replace(w, chains=[c]))
        ps.set_counts(0, dev_counts(cnts[i]))
        l1, g1, b1 = ps.value_and_grad(dev(nus[i].ravel()), dev(c.bias[None]))
        o = pb.offsets[i]
        assert torch.equal(lb[i:i + 1], l1)
        assert torch.equal(gb[o:o + c.n ** 3], g1)
        assert torch.equal(bb[i:i + 1], b1)


def test_rejects_unsupported_mesh():
    from paper_2506_03969_amd import FzwError
    w = fi.small_variant(fi.workload("c0"), 16)
    w.chains[0].n = 100
    with pytest.raises(FzwError, match="status -2"):
        plan_for(w)


@pytest.mark.parametrize("rsd", [None, RADIAL], ids=["los", "radial"])
def test_cic_methods_bit_identical(rsd):
    """The sorted-gather deposit and the fixed-point atomic deposit give the
    same density bit for bit (same FP32 weights, exact integer sums)."""
    w, m, nu, counts, p, bias, b = _gpu_forward("c2", 64, "near", rsd=rsd)
    x = dev(nu.ravel())
    l1 = p.forward(x, bias).clone()
    r1 = p.get_field(0, 4).clone()
    p.set_cic_method("atomic")
    l2 = p.forward(x, bias).clone()
    r2 = p.get_field(0, 4).clone()
    p.set_cic_method("sorted")
    assert torch.equal(r1, r2)
    assert torch.equal(l1, l2)


@pytest.mark.parametrize("case", [("c0fd", None), ("c2", 32), ("c2", 96)], ids=_ids)
def test_wiener_start_matches_oracle(case):
    """The Wiener-filter starting point (fzw_wiener_start) against the
    oracle's, element by element (relative 1e-5 normwise), on one chain and on
    a plan of two meshes."""
    from oracle import wiener
    name, n = case
    w, m, nu_t, nu_e, counts = mock_case(name, n)
    p = plan_for(w)
    p.set_counts(0, dev_counts(counts))
    got = host(p.wiener_start()).reshape(counts.shape)
    ref = wiener.wiener_white_noise(m, counts)
    err = relnorm(got, ref)
    print(name, n, "wiener start err %.2e, |nu| rms %.3f" % (err, float(np.sqrt(np.mean(ref ** 2)))))
    assert err < 1e-5


@pytest.mark.parametrize("case", [("c2", 64), ("c1", None)], ids=_ids)
def test_validation_statistics_match_oracle(case):
    """Power-spectrum monopole and quadrupole (redshift-space density), cross
    spectrum with the linear density, and the reduced bispectrum at
    k1 = 0.1, k2 = 0.2 h/Mpc, through the C ABI against the oracle's
    statistics of the same FP32 fields.  Mode counts and triangle counts are
    exact; spectra within 1e-5 relative; bispectra within 1e-4 of their
    largest magnitude."""
    from oracle import stats
    name, n = case
    w, m, nu, counts, p, bias, b = _gpu_forward(name, n, "near")
    st = m.forward(nu, b, counts)
    ch = w.chains[0]
    delta = (st["rho"] - 1.0).astype(np.float32)
    dl = st["dl"].astype(np.float32)
    kf = 2 * np.pi / ch.box
    nb = 12
    gp = host(p.power_multipoles(dev(delta.ravel()), None, k_lo=kf, dk=2 * kf, nbins=nb, mesh_n=ch.n))
    km, cnt, p0, p2 = stats.multipoles(delta.astype(np.float64), None, ch.box, kf, 2 * kf, nb)
    assert np.array_equal(gp[:, 1], cnt)
    assert np.allclose(gp[:, 0], km, rtol=1e-12)
    assert np.allclose(gp[:, 2], p0, rtol=1e-5)
    assert np.all(np.abs(gp[:, 3] - p2) < 1e-5 * np.abs(p0))
    gx = host(p.power_multipoles(dev(delta.ravel()), dev(dl.ravel()), k_lo=kf, dk=2 * kf, nbins=nb, mesh_n=ch.n))
    _, _, x0, x2 = stats.multipoles(delta.astype(np.float64), dl.astype(np.float64), ch.box, kf, 2 * kf, nb)
    assert np.allclose(gx[:, 2], x0, rtol=1e-5, atol=1e-5 * np.abs(x0).max())
    thetas = np.linspace(0.05, np.pi - 0.05, 9)
    gb = host(p.bispectrum(dev(delta.ravel()), 0.1, 0.2, 2 * kf, thetas, mesh_n=ch.n))
    k3, b, q, tri = stats.bispectrum(delta.astype(np.float64), ch.box, 0.1, 0.2, 2 * kf, thetas)
    print(name, n, "P0 err %.2e  B max err %.2e (max |B| %.3e)  Q" % (
        float(np.max(np.abs(gp[:, 2] / p0 - 1))), float(np.max(np.abs(gb[:, 1] - b))), float(np.abs(b).max())),
        np.round(gb[:, 2], 4), np.round(q, 4))
    assert np.allclose(gb[:, 0], k3, rtol=1e-12)
    assert np.allclose(gb[:, 3], tri, rtol=1e-5)
    assert np.all(np.abs(gb[:, 1] - b) < 1e-4 * np.abs(b).max())
    assert np.all(np.abs(gb[:, 2] - q) < 1e-4 * np.abs(q).max())
