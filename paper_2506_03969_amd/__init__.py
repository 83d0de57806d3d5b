"""MI355X (gfx950) implementation of the differentiable fuzzy-cosmic-web
field-level likelihood: forward model, hand-written adjoint, leapfrog and NUTS behind
the C ABI of include/fzw.h, with a thin PyTorch binding (fzw.py)."""
from .fzw import (CosmoParams, DualAveraging, FIELD_DPSI, FIELD_DRHO, FzwError, LogLikelihood, NF_GRAD,
                  NF_HAMILTONIAN, NF_LOGL, NF_STATE, NUTS_MAX_DEPTH, Plan, RSD_RADIAL, WebParams, WEB_DELTA,
                  WEB_PHI, fft_schedule, load_library, nuts_n_uniforms, set_fft_schedule)

__all__ = ["CosmoParams", "DualAveraging", "FIELD_DPSI", "FIELD_DRHO", "FzwError", "LogLikelihood", "NF_GRAD",
           "NF_HAMILTONIAN", "NF_LOGL", "NF_STATE", "NUTS_MAX_DEPTH", "Plan", "RSD_RADIAL",
           "WebParams", "WEB_DELTA", "WEB_PHI", "fft_schedule", "load_library", "nuts_n_uniforms",
           "set_fft_schedule"]
