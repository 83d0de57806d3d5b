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
def mock_case(name, n=None, tau_sc=None, chain=0):
    """(workload, oracle model, truth nu, eval nu, counts) for a workload."""
    kw = {"tau_sc": tau_sc} if tau_sc is not None else {}
    w = workload_at(name, n, **kw)
    ch = w.chains[chain]
    m = oracle_model(w, chain)
    nu_t = fi.white_noise(ch, fi.ROLE_TRUTH_NU)
    rng = fi.rng_for(ch, fi.ROLE_DATA)
    counts, _ = make_counts(m, nu_t, ch.bias, ch.mean_count,
                            lambda nb, b: fi.gamma_poisson_counts(nb, b, rng))
    nu_e = fi.white_noise(ch, fi.ROLE_EVAL_NU)
    return w, m, nu_t, nu_e, counts
