"""Shared test helpers: oracle models and mock data for the named workloads."""
import functools

import numpy as np

import fzw_inputs as fi
from oracle.mock import make_counts
from oracle.model import Model, Settings


def workload_at(name, n=None, **cosmo_kw):
    w = fi.workload(name)
    if n is not None and n != w.chains[0].n:
        w = fi.small_variant(w, n)
    if cosmo_kw:
        import dataclasses
        w = dataclasses.replace(w, cosmo=dataclasses.replace(w.cosmo, **cosmo_kw))
    return w


def oracle_model(w, chain=0):
    return Model(Settings.from_workload(w.cosmo, w.web, w.chains[chain]))


@functools.lru_cache(maxsize=16)
def mock_case(name, n=None, tau_sc=None, chain=0, rsd_axis=None):
    """(workload, oracle model, truth nu, eval nu, counts) for a workload."""
    kw = {"tau_sc": tau_sc} if tau_sc is not None else {}
    if rsd_axis is not None:
        kw["rsd_axis"] = rsd_axis
    w = workload_at(name, n, **kw)
    ch = w.chains[chain]
    m = oracle_model(w, chain)
    nu_t = fi.white_noise(ch, fi.ROLE_TRUTH_NU)
    rng = fi.rng_for(ch, fi.ROLE_DATA)
    counts, _ = make_counts(m, nu_t, ch.bias, ch.mean_count,
                            lambda nb, b: fi.gamma_poisson_counts(nb, b, rng))
    nu_e = fi.white_noise(ch, fi.ROLE_EVAL_NU)
    return w, m, nu_t, nu_e, counts


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


def oracle_floor(m, nu, bias, counts, ref_dnu, ref_db):
    """How far the FP64 gradient itself moves when its input is rounded to FP32
    or perturbed at relative 5e-7 (the size of the error an FP32 path
    accumulates over its ~10 FFT passes: its forward fields carry 2-9e-7):
    the conditioning floor of any FP32 path.  Returns (d/dnu normwise, bias
    per-entry) sensitivities."""
    rng = np.random.default_rng(99)
    fn, fb = 0.0, 0.0
    # a few samples: the largest moves come from rare events (a particle
    # crossing a CIC cell face next to a tracer-holding, nearly empty cell)
    samples = [nu.astype(np.float32).astype(np.float64)]
    samples += [nu * (1 + 5e-7 * rng.standard_normal(nu.shape)) for _ in range(4)]
    for x in samples:
        _, g, b = m.value_and_grad(x, bias, counts)
        fn = max(fn, relnorm(g, ref_dnu))
        fb = max(fb, bias_entry_error(b, ref_db))
    return fn, fb
