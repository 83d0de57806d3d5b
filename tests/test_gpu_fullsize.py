"""Parity and invariants at the full workload sizes, in the launch
configuration the benchmark times.

* 256^3 two-web workload: fields, log-likelihood and both gradients against
  the FP64 oracle at a near-truth state.
* Ragged batch (one 64^3, one 96^3 and one 128^3 chain in one plan, as in the
  32-chain workload): every chain against the oracle, and a batched leapfrog
  trajectory equal bit for bit to the per-chain trajectories.
* 512^3 trajectory workload: the forward stages the oracle finishes in a
  test's time (delta_L, Psi, the redshift-space density and both webs'
  tensors) against the oracle; the rest through properties that hold at any
  size: the transform against numpy, mass conservation of the deposit,
  determinism, agreement of the two likelihood paths, and central differences
  of the FP64-reduced logL along the gradient (1e-3), a random bias direction
  (1e-3) and a random direction of nu (sign and size).
"""
import dataclasses
import os
import sys

import numpy as np
import pytest

import fzw_inputs as fi
from tests.helpers import FIELD_TOL, GRAD_TOL, LOGL_TOL, Floor, fp32, mock_case, off_face, oracle_gradient

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

if not torch.cuda.is_available():  # pragma: no cover - collected on CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)

from tests.gpu_helpers import bias_entry_error, dev, dev_counts, host, plan_for, relnorm  # noqa: E402

def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class _C2:
    """The 256^3 two-web workload at a state near the data's noise, on the
    same float32 inputs as the oracle; the GPU results are taken once, the
    oracle's stages in the tests that use them (each test stays well under
    three minutes on 16 host threads)."""

    def __init__(self):
        from oracle import model as om
        from paper_2506_03969_amd import FIELD_DPSI, FIELD_DRHO
        om.set_workers(16)
        _say("c2 256^3: mock data (oracle forward at truth)")
        w, m, nu_t, nu_e, counts = mock_case("c2")
        ch = w.chains[0]
        self.m, self.counts = m, counts
        self.nu = fp32(fi.near_truth_noise(ch))
        self.b = fp32(ch.bias)
        p = plan_for(w)
        p.set_counts(0, dev_counts(counts))
        nu, bias = dev(self.nu.ravel()), dev(self.b[None])
        logl, dnu, dbias = p.value_and_grad(nu, bias)
        self.g = (float(host(logl)[0]), host(dnu).reshape(self.nu.shape), host(dbias).reshape(self.b.shape))
        lf, nbar = p.forward(nu, bias, want_nbar=True)
        self.g_lf = float(host(lf)[0])
        self.fields = {"dl": host(p.get_field(0, 0)), "rho": host(p.get_field(0, 4)),
                       "f": np.exp(host(p.get_field(0, 5)).ravel()), "nbar": host(nbar),
                       "psi": np.stack([host(p.get_field(0, k)) for k in (1, 2, 3)]),
                       "T": [np.stack([host(p.get_field(0, 6 + 6 * wi + k)) for k in range(6)]) for wi in range(2)]}
        _say("c2 256^3: oracle forward")
        self.st = m.forward(self.nu, self.b, counts)
        # conditioned data: no tracer where the density is below 0.05 of the mean
        cc = counts.copy().reshape(-1)
        cc[self.st["x"] < 0.05] = 0
        self.cc = cc.reshape(counts.shape)
        p.set_counts(0, dev_counts(self.cc))
        logl, dnu, dbias = p.value_and_grad(nu, bias)
        self.gc = (float(host(logl)[0]), host(dnu).reshape(self.nu.shape), host(dbias).reshape(self.b.shape),
                   host(p.get_field(0, FIELD_DRHO)), np.stack([host(p.get_field(0, FIELD_DPSI + j)) for j in range(3)]))
        self.ref = None
        self.refc = None


@pytest.fixture(scope="module")
def c2():
    return _C2()


@pytest.mark.timeout(170)
def test_c2_full_size_fields_and_logl(c2):
    """256^3 (the bench workload): every forward intermediate within 1e-5
    normwise of the oracle, logL within 1e-4, and forward and gradient calls
    give the same logL bit for bit."""
    gpu, st = c2.fields, c2.st
    errs = {"delta_L": relnorm(gpu["dl"], st["dl"]), "psi": relnorm(gpu["psi"], st["psi"]),
            "rho": relnorm(gpu["rho"], st["rho"]), "f": relnorm(gpu["f"], st["f"]),
            "nbar": relnorm(gpu["nbar"], st["nbar"])}
    for wi in range(2):
        errs["T%d" % wi] = relnorm(gpu["T"][wi], np.stack(st["tens"][wi]))
    errs["logL"] = abs(c2.g[0] - st["logl"]) / abs(st["logl"])
    _say("c2 256^3 fields:", " ".join("%s=%.2e" % kv for kv in errs.items()))
    c2.fields = None
    assert c2.g[0] == c2.g_lf
    for k, v in errs.items():
        assert v < (LOGL_TOL if k == "logL" else FIELD_TOL), (k, v)


@pytest.mark.timeout(170)
def test_c2_full_size_gradient(c2):
    """256^3, the mock data as drawn: the bias gradient within 1e-4 normwise
    and per entry, d logL/d nu within 1e-4 or ten times the conditioning floor
    (tracers in nearly empty cells, whose terms scale as 1/x^2, set it)."""
    _say("c2 256^3: oracle adjoint")
    ref_dnu, ref_db = c2.m.adjoint(c2.st)
    _, g_dnu, g_db = c2.g
    e_nu, e_bn, e_b = relnorm(g_dnu, ref_dnu), relnorm(g_db, ref_db), bias_entry_error(g_db, ref_db)
    _say("c2 256^3 gradient, data as drawn: dnu=%.2e dbias norm=%.2e entry=%.2e" % (e_nu, e_bn, e_b))
    assert np.all(np.isfinite(g_dnu)) and np.all(np.isfinite(g_db))
    assert e_bn < GRAD_TOL and e_b < GRAD_TOL
    fl = Floor(c2.m, c2.nu, c2.b, c2.counts, ref_dnu, ref_db, c2.st["dbias_abs"])
    ok = fl.holds_nu(e_nu)
    _say("c2 256^3 floor, data as drawn (%d draws): nu %.2e" % (fl.draws, fl.nu_f))
    c2.st = None
    assert ok


@pytest.mark.timeout(170)
def test_c2_full_size_conditioned_cotangents(c2):
    """256^3, conditioned data (those tracers removed): d logL/d rho (every
    voxel) and d logL/d Psi (particles more than 1e-5 cells from every cell
    face) at the fixed 1e-4, logL 1e-4, bias gradient 1e-4 normwise; d logL/d
    nu within 1e-4 or ten times the floor (about a thousand particles lie
    within float32 noise of a cell face at this size)."""
    _say("c2 256^3: oracle on the conditioned data (%d tracers removed)" % int(c2.counts.sum() - c2.cc.sum()))
    st = c2.m.forward(c2.nu, c2.b, c2.cc)
    ref_dnu, ref_db = c2.m.adjoint(st)
    fl = Floor(c2.m, c2.nu, c2.b, c2.cc, ref_dnu, ref_db, st["dbias_abs"])
    c2.refc = fl
    g_l, g_dnu, g_db, g_drho, g_dpsi = c2.gc
    keep = off_face(st["pos"])
    e = {"logL": abs(g_l - st["logl"]) / abs(st["logl"]), "dnu": relnorm(g_dnu, ref_dnu),
         "drho": relnorm(g_drho, st["drho"]),
         "dpsi_off_face": relnorm(g_dpsi.reshape(3, -1)[:, keep], st["dpsi"].reshape(3, -1)[:, keep]),
         "dbias": relnorm(g_db, ref_db), "dbias_entry": bias_entry_error(g_db, ref_db)}
    _say("c2 256^3 conditioned (%d particles near a face):" % int((~keep).sum()),
         " ".join("%s=%.2e" % kv for kv in e.items()))
    assert e["logL"] < LOGL_TOL
    assert e["drho"] < GRAD_TOL and e["dpsi_off_face"] < GRAD_TOL
    assert e["dbias"] < GRAD_TOL
    del st
    ok = fl.holds_nu(e["dnu"])
    _say("c2 256^3 conditioned d/dnu floor (%d draws): %.2e" % (fl.draws, fl.nu_f))
    assert ok


@pytest.mark.timeout(170)
def test_c2_full_size_conditioned_bias_entries(c2):
    """256^3, conditioned data: each bias-table entry within 1e-4 or ten times
    the conditioning floor (entries whose voxel sums cancel)."""
    if c2.refc is None:
        pytest.skip("needs test_c2_full_size_conditioned_cotangents")
    fl = c2.refc
    g_db = c2.gc[2]
    e_b = bias_entry_error(g_db, fl.args[5])
    fl_ok = fl.holds_bias(g_db)
    _say("c2 256^3 conditioned bias entries %.2e (floor %d draws: %.2e)" % (e_b, fl.draws, fl.bias_f))
    assert fl_ok


def _ragged():
    w = fi.workload("c3")
    sel = [0, 12, 22]                      # 64^3, 96^3, 128^3
    return w, sel


@pytest.mark.timeout(600)
def test_ragged_batch_against_oracle():
    """One plan holding a 64^3, a 96^3 and a 128^3 chain (the mix of the
    32-chain workload): each chain's logL and gradients against the oracle."""
    from oracle import model as om
    om.set_workers(16)
    w, sel = _ragged()
    cases = []
    for c in sel:
        _say("ragged: mock data for chain", c, "n =", w.chains[c].n)
        ww, m, nu_t, nu_e, counts = mock_case("c3", None, None, c)
        ch = ww.chains[c]
        cases.append((ch, m, fp32(fi.near_truth_noise(ch)), counts, fp32(ch.bias)))
    p = plan_for(w, sel)
    for i, (ch, m, nu, counts, b) in enumerate(cases):
        p.set_counts(i, dev_counts(counts))
    nu_all = dev(np.concatenate([nu.ravel() for _, _, nu, _, _ in cases]))
    bias_all = dev(np.stack([b for _, _, _, _, b in cases]))
    logl, dnu, dbias = p.value_and_grad(nu_all, bias_all)
    gl, gd, gb = host(logl), host(dnu), host(dbias)
    for i, (ch, m, nu, counts, b) in enumerate(cases):
        ref_l, ref_dnu, ref_db, st = oracle_gradient(m, nu, b, counts)
        o = p.offsets[i]
        g = gd[o:o + ch.n ** 3].reshape(nu.shape)
        e_l = abs(gl[i] - ref_l) / abs(ref_l)
        e_nu = relnorm(g, ref_dnu)
        e_bn = relnorm(gb[i], ref_db)
        e_b = bias_entry_error(gb[i], ref_db)
        fl = Floor(m, nu, b, counts, ref_dnu, ref_db, st["dbias_abs"])
        ok_nu, ok_b = fl.holds_nu(e_nu), fl.holds_bias(gb[i])
        _say("ragged chain n=%d: logL=%.2e dnu=%.2e dbias norm=%.2e entry=%.2e (floor %d draws: nu %.2e bias %.2e)"
             % (ch.n, e_l, e_nu, e_bn, e_b, fl.draws, fl.nu_f, fl.bias_f))
        assert e_l < LOGL_TOL
        assert e_bn < GRAD_TOL and ok_nu and ok_b


@pytest.mark.timeout(600)
def test_ragged_leapfrog_equals_per_chain():
    """A graph-captured trajectory of the ragged batch moves every chain
    exactly as a plan holding that chain alone does (bit for bit)."""
    w, sel = _ragged()
    chains = [w.chains[c] for c in sel]
    wsel = dataclasses.replace(w, chains=chains)
    mu, sig = fi.prior_arrays(w)
    tie = fi.tie_array(w)
    counts = [fi.timing_counts(ch) for ch in chains]
    nus = [fi.white_noise(ch, fi.ROLE_EVAL_NU).astype(np.float32) for ch in chains]
    g = np.random.default_rng(3)
    pnus = [g.standard_normal(x.shape).astype(np.float32) for x in nus]
    us = [fi.free_start(w, ch).astype(np.float32) for ch in chains]
    pus = [g.standard_normal(u.shape).astype(np.float32) for u in us]
    steps, eps = 3, 1e-3

    def run(idx):
        ww = dataclasses.replace(wsel, chains=[chains[i] for i in idx])
        p = plan_for(ww)
        p.set_sampling(tie, mu, sig)
        for k, i in enumerate(idx):
            p.set_counts(k, dev_counts(counts[i]))
        nu = dev(np.concatenate([nus[i].ravel() for i in idx]))
        pn = dev(np.concatenate([pnus[i].ravel() for i in idx]))
        u = dev(np.stack([us[i] for i in idx]))
        pu = dev(np.stack([pus[i] for i in idx]))
        base = dev(np.stack([chains[i].bias for i in idx]))
        minv = torch.ones_like(nu)
        minv_u = torch.full_like(u, 1e-2)
        step = dev(np.full(len(idx), eps))
        h0, h1 = p.leapfrog(nu, u, pn, pu, base, minv, minv_u, step, steps)
        return p, host(nu), host(u), host(h0), host(h1)

    pb, nu_b, u_b, h0_b, h1_b = run([0, 1, 2])
    _say("ragged leapfrog H0", h0_b, "H1", h1_b)
    assert np.all(np.isfinite(h1_b))
    for i in range(3):
        ps, nu_s, u_s, h0_s, h1_s = run([i])
        o = pb.offsets[i]
        n3 = chains[i].n ** 3
        assert np.array_equal(nu_b[o:o + n3], nu_s[:n3])
        assert np.array_equal(u_b[i], u_s[0])
        assert h0_b[i] == h0_s[0] and h1_b[i] == h1_s[0]


@pytest.mark.timeout(900)
def test_512_invariants():
    """512^3 (the 20-step trajectory workload): transform against numpy, mass
    conservation, determinism, likelihood paths, directional derivative."""
    import scipy.fft as sfft
    w = fi.workload("c4")
    ch = w.chains[0]
    n = ch.n
    p = plan_for(w)
    _say("512^3: transform against numpy")
    rng = np.random.default_rng(512)
    x = rng.standard_normal((n, n, n)).astype(np.float32)
    got = p.fft_r2c(dev(x[None]))[0]
    ref = sfft.rfftn(x.astype(np.float64), workers=16)
    err = relnorm(got.cpu().numpy(), ref)
    back = host(p.fft_c2r(got[None]))[0]
    err2 = relnorm(back, x.astype(np.float64) * float(n) ** 3)
    _say("512^3 fft r2c err=%.2e round trip err=%.2e" % (err, err2))
    del got, ref, back
    assert err < 2e-6 and err2 < 4e-6

    _say("512^3: likelihood and gradient")
    # data drawn from the model's own mean at the truth noise, and the check
    # made at that noise (a self-consistency check: nothing here is compared
    # with the oracle).  Away from it, e.g. at a 5% perturbation, tracers fall
    # in cells that are nearly empty there, log f ~ -rho_th / x makes d/dx
    # ~ 1/x^2 huge, and no finite step sees the first-order change (the 256^3
    # gradient, which matches the oracle, behaves the same way there).
    #
    # A second plan runs the likelihood pass in float64 per voxel.  The mean
    # the data are drawn from is that plan's, so that the data do not depend
    # on the default pass's rounding: the Poisson sampler takes a variable
    # number of uniforms per voxel, and one changed mean re-draws every voxel
    # after it.
    os.environ["FZW_LIKELIHOOD_FP64"] = "1"
    try:
        p64 = plan_for(w)
    finally:
        os.environ.pop("FZW_LIKELIHOOD_FP64", None)
    nu = dev(fi.white_noise(ch, fi.ROLE_TRUTH_NU).astype(np.float32).ravel())
    bias = dev(ch.bias[None])
    for q in (p, p64):
        q.set_counts(0, dev_counts(fi.timing_counts(ch)))
    _, nbar = p64.forward(nu, bias, want_nbar=True)
    nbar_h = host(nbar).reshape((n,) * 3)
    counts = fi.gamma_poisson_counts(nbar_h, np.full_like(nbar_h, float(ch.bias[0, fi.COL_BETA])),
                                     fi.rng_for(ch, fi.ROLE_DATA))
    del nbar, nbar_h
    for q in (p, p64):
        q.set_counts(0, dev_counts(counts))
    l1, g1, b1 = [t.clone() for t in p.value_and_grad(nu, bias)]
    # the float32 likelihood pass against the float64 one on the same data:
    # the gradients agree to float32 rounding, and so does the change of lnP
    # between two bias tables 1e-4 apart (what a Metropolis decision sees;
    # rounding shared by all voxels of one beta would show here as O(1))
    l64, g64, b64 = p64.value_and_grad(nu, bias)
    e_l = abs(float(l1[0]) - float(l64[0])) / abs(float(l64[0]))
    e_g = float((g1.double() - g64.double()).norm() / g64.double().norm())
    e_b = float((b1.double() - b64.double()).norm() / b64.double().norm())
    _say("512^3 float32 vs float64 likelihood pass: logL %.2e grad %.2e bias grad %.2e" % (e_l, e_g, e_b))
    assert e_l < 1e-6 and e_g < 1e-5 and e_b < 1e-4
    rb = torch.from_numpy(np.random.default_rng(7).standard_normal(tuple(bias.shape)).astype(np.float32)).cuda()
    bias2 = bias * (1 + 1e-4 * rb)
    d32 = float(p.forward(nu, bias2)[0]) - float(l1[0])
    d64 = float(p64.forward(nu, bias2)[0]) - float(l64[0])
    _say("512^3 change of logL over a 1e-4 bias move: float32 pass %.6e float64 pass %.6e" % (d32, d64))
    assert abs(d32 - d64) < 0.05
    del p64, l64, g64, b64
    rho = p.get_field(0, 4).double()
    mass = float(rho.sum())
    del rho
    l2, g2, b2 = p.value_and_grad(nu, bias)
    lf = p.forward(nu, bias)
    _say("512^3 logL=%.9e forward=%.9e mass rel err=%.2e" % (float(l1[0]), float(lf[0]), abs(mass - n ** 3) / n ** 3))
    assert abs(mass - float(n) ** 3) < 1e-6 * float(n) ** 3
    assert torch.equal(l1, l2) and torch.equal(g1, g2) and torch.equal(b1, b2)
    assert float(lf[0]) == float(l1[0])
    assert bool(torch.isfinite(g1).all()) and bool(torch.isfinite(b1).all())

    # directional derivatives: central differences of the FP64-reduced logL.
    # Along the gradient the direction concentrates on the stiffest voxels and
    # the O(h^2) truncation of a central difference at h = 1e-2 reaches ~1e-3
    # relative, so the differences at h and h/2 are Richardson-extrapolated
    # (error O(h^4)).
    gd = g1 / g1.norm()

    def central(h):
        return (float(p.forward(nu + h * gd, bias)[0]) - float(p.forward(nu - h * gd, bias)[0])) / (2 * h)

    h = 1e-2
    fd1, fd2 = central(h), central(h / 2)
    fd = (4.0 * fd2 - fd1) / 3.0
    an = float(g1.double().norm())
    _say("512^3 along the gradient: FD(h) %.6e FD(h/2) %.6e extrapolated %.6e adjoint %.6e rel %.2e"
         % (fd1, fd2, fd, an, abs(fd - an) / abs(an)))
    assert abs(fd - an) < 1e-3 * abs(an)
    # along a random direction of nu the check is only coarse: the forward
    # logL carries FP32 noise of ~2e-9 relative (~0.4 of 1.7e8), i.e. ~2e2 on a
    # central difference with h = 1e-3, against a directional derivative of
    # ~5e3; and the derivative itself is ill-conditioned at this size (a few
    # tracers sit in cells with nbar << 1, where d logL / dx ~ 1/x^2: the
    # tables and the closed-form multipliers, equal to ~1e-7, give values 20%
    # apart).  Sign and magnitude are held.
    d = torch.from_numpy(np.random.default_rng(5).standard_normal(n ** 3).astype(np.float32)).cuda()
    h = 1e-3
    fd = (float(p.forward(nu + h * d, bias)[0]) - float(p.forward(nu - h * d, bias)[0])) / (2 * h)
    an = float(torch.dot(g1.double(), d.double()))
    _say("512^3 random direction: FD %.6e adjoint %.6e rel %.2e" % (fd, an, abs(fd - an) / abs(an)))
    assert abs(fd - an) < 0.25 * abs(an)
    # along a random relative change of the bias table the likelihood is
    # smooth and the difference converges: held to 1e-3 (a step of 1e-3
    # keeps the float32 noise of the forward logL, ~3e-3, well below the
    # difference, ~16)
    rb = torch.from_numpy(np.random.default_rng(6).standard_normal(tuple(bias.shape)).astype(np.float32)).cuda() * bias
    hb = 1e-3
    fdb = (float(p.forward(nu, bias + hb * rb)[0]) - float(p.forward(nu, bias - hb * rb)[0])) / (2 * hb)
    anb = float(torch.sum(b1.double() * rb.double()))
    _say("512^3 random bias direction: FD %.6e adjoint %.6e rel %.2e" % (fdb, anb, abs(fdb - anb) / abs(anb)))
    assert abs(fdb - anb) < 1e-3 * abs(anb)


class _C4:
    """The 512^3 trajectory workload (two webs, redshift space along z) at a
    state near the data's noise: the GPU's forward intermediates, taken once,
    against the FP64 oracle's stages, computed in the tests that use them."""

    def __init__(self):
        from oracle import model as om
        from tests.helpers import oracle_model
        om.set_workers(16)
        w = fi.workload("c4")
        ch = w.chains[0]
        self.n = ch.n
        self.nu = fp32(fi.near_truth_noise(ch))
        self.b = fp32(ch.bias)
        _say("c4 512^3: GPU forward")
        p = plan_for(w)
        p.set_counts(0, dev_counts(fi.timing_counts(ch)))
        p.forward(dev(self.nu.ravel()), dev(self.b[None]))
        torch.cuda.synchronize()
        get = lambda k: p.get_field(0, k).cpu().numpy().reshape((self.n,) * 3)
        self.gpu = {"dl": get(0), "psi": np.stack([get(k) for k in (1, 2, 3)]), "rho": get(4),
                    "T": [np.stack([get(6 + 6 * wi + k) for k in range(6)]) for wi in range(2)]}
        del p
        torch.cuda.empty_cache()
        self.m = oracle_model(w, 0)
        self.psi = None


@pytest.fixture(scope="module")
def c4():
    return _C4()


@pytest.mark.timeout(170)
def test_c4_full_size_lpt_stages(c4):
    """512^3: delta_L (the white-noise filter in the 512 mixing pass) and Psi
    (the six LPT Hessians, the spherical-collapse term and the ALPT blend
    through the 512 passes) within 1e-5 normwise of the oracle on the same
    float32 white noise."""
    _say("c4 512^3: oracle delta_L and ALPT")
    m = c4.m
    psi, lpt = m.alpt(m.linear_density_hat(c4.nu.astype(np.float64)))
    e_dl = relnorm(c4.gpu["dl"], lpt["dl"])
    del lpt
    e_psi = relnorm(c4.gpu["psi"], psi)
    c4.psi = psi
    c4.gpu["dl"] = c4.gpu["psi"] = None
    _say("c4 512^3 fields: delta_L=%.2e psi=%.2e" % (e_dl, e_psi))
    assert e_dl < FIELD_TOL and e_psi < FIELD_TOL


@pytest.mark.timeout(170)
def test_c4_full_size_density_and_tensors(c4):
    """512^3: the redshift-space density of the sorted deposit (134M
    particles) and both webs' tensors within 1e-5 normwise of the oracle's,
    which start from the oracle's own displacement."""
    if c4.psi is None:
        pytest.skip("needs the oracle displacement of test_c4_full_size_lpt_stages")
    m = c4.m
    _say("c4 512^3: oracle positions and deposit")
    rho = m.cic(m.positions(c4.psi))
    c4.psi = None
    e_rho = relnorm(c4.gpu["rho"], rho)
    _say("c4 512^3 rho=%.2e; oracle web tensors" % e_rho)
    tens = m.web_tensors(m.g.rfft(rho - 1.0))
    del rho
    e_t = [relnorm(c4.gpu["T"][wi], np.stack(tens[wi])) for wi in range(2)]
    _say("c4 512^3 fields: rho=%.2e T0=%.2e T1=%.2e" % (e_rho, e_t[0], e_t[1]))
    assert e_rho < FIELD_TOL and max(e_t) < FIELD_TOL
