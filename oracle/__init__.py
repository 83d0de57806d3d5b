"""FP64 CPU oracle of the differentiable fuzzy-cosmic-web likelihood.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything here; only the tests, the
smoke check and the benchmark's CPU-baseline leg use it.  It shares no code,
tables or constants with the GPU path.

Plain NumPy/SciPy in float64, written stage by stage from the paper:
  cosmology.py  linear power spectrum (BBKS shape, sigma8 normalisation) and the
                white-noise filter of Appendix A
  model.py      forward model (Appendix A, Section 2.3 ALPT, CIC, Section 2.9 RSD,
                Section 2.8 fuzzy web, Section 2.6 bias, Section 2.7 likelihood)
                and its hand-written adjoint
  hmc.py        potential, Hamiltonian and leapfrog (Sections 2.1-2.2)
  nuts.py       the no-U-turn transition, dual averaging and Welford variances
                used by the warm-up (Section 2.2, after the published method)
  wiener.py     the Wiener-filter starting point of the chains (Section 2.2)
  stats.py      binned power-spectrum estimator (a test tool)
  mock.py       mock data from the forward model (Section 3 recipe)

Parity status: every stage is pinned by closed forms, limits or library
routines in tests/test_oracle_*.py, except the readings listed as
"parity unpinned" in the docstrings of model.py (the BBKS coefficients beyond
their limits, the delta-web sign/scale reading and the signed-epsilon bias
reading); the paper prints no intermediate value to pin those against.
"""
