"""Both FFT kernel families of every pass type (register four-step and LDS
Stockham for the z and mixing x/y passes; persistent four-step or the mixing
kernel for pure x/y transforms), forced one combination at a time: each
transform against numpy, and the log-likelihood and gradients of a two-web
case against the FP64 oracle.  At 96 only the mixing x/y passes have two
families (the four-step one splits a line into three 32-point sub-lines)."""
import itertools

import numpy as np
import pytest

import fzw_inputs as fi

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from tests.gpu_helpers import dev, dev_counts, host, plan_for, relnorm  # noqa: E402
from tests.helpers import GRAD_TOL, LOGL_TOL, Floor, fp32, mock_case  # noqa: E402

COMBOS = list(itertools.product(("four-step", "stockham"), ("four-step", "stockham"), ("four-step", "mixing")))


@pytest.mark.parametrize("n", [32, 64, 96, 128])
def test_every_fft_family(n):
    """Each combination against numpy (transforms) and against the FP64
    oracle on the same float32 inputs (logL 1e-4, bias gradient 1e-4
    normwise; d/dnu within 1e-4 or ten times the oracle's own conditioning
    floor: the rule of the parity tests)."""
    from paper_2506_03969_amd import fft_schedule, set_fft_schedule
    w, m, nu_t, nu_e, counts = mock_case("c2", n)
    ch = w.chains[0]
    nu_h = fp32(fi.near_truth_noise(ch))
    b_h = fp32(ch.bias)
    p = plan_for(w)                        # tunes the schedule of this size
    tuned = fft_schedule(n)
    print("n=%d tuned:" % n, {k: "%s (%.1f / %.1f us)" % v for k, v in tuned.items()})
    p.set_counts(0, dev_counts(counts))
    nu = dev(nu_h.ravel())
    bias = dev(b_h[None])
    ref_l, ref_dnu, ref_db = m.value_and_grad(nu_h, b_h, counts)
    fl = Floor(m, nu_h, b_h, counts, ref_dnu, ref_db)
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, n, n)).astype(np.float32)
    ref_k = np.fft.rfftn(x.astype(np.float64))
    try:
        for z, xy, pure in COMBOS:
            set_fft_schedule(n, z, xy, pure)
            got = p.fft_r2c(dev(x[None]))
            e1 = relnorm(got[0].cpu().numpy(), ref_k)
            e2 = relnorm(host(p.fft_c2r(got))[0], x.astype(np.float64) * n ** 3)
            l, g, b = p.value_and_grad(nu, bias)
            el = abs(float(l[0]) - ref_l) / abs(ref_l)
            eg = relnorm(host(g).reshape(nu_h.shape), ref_dnu)
            eb = relnorm(host(b).reshape(ref_db.shape), ref_db)
            print("n=%d z=%s xy=%s pure=%s: r2c %.1e c2r %.1e | vs oracle: logL %.1e dnu %.1e dbias %.1e" % (
                n, z, xy, pure, e1, e2, el, eg, eb))
            assert e1 < 2e-6 and e2 < 2e-6
            assert el < LOGL_TOL and eb < GRAD_TOL
            assert fl.holds_nu(eg), (eg, fl.nu_f)
    finally:
        set_fft_schedule(n, tuned["z"][0], tuned["xy"][0], tuned["pure"][0])
