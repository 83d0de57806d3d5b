"""MI355X (gfx950) implementation of the differentiable fuzzy-cosmic-web
field-level likelihood: forward model, hand-written adjoint and leapfrog behind
the C ABI of include/fzw.h, with a thin PyTorch binding (fzw.py)."""
from .fzw import (CosmoParams, FzwError, LogLikelihood, Plan, WebParams, WEB_DELTA, WEB_PHI, fft_schedule,
                  load_library, set_fft_schedule)

__all__ = ["CosmoParams", "FzwError", "LogLikelihood", "Plan", "WebParams", "WEB_DELTA", "WEB_PHI",
           "fft_schedule", "load_library", "set_fft_schedule"]
