"""Python binding of libfzw.so (the gfx950 HIP library behind include/fzw.h).

Argument marshalling only: every stage of the forward model, its adjoint and
the leapfrog runs in the library's HIP kernels.  PyTorch provides the device
memory (tensors on cuda) and the stream (the current torch stream at plan
creation).  There is no CPU fallback: without the built library or a GPU the
calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfzw.so")
_lib = None

WEB_PHI, WEB_DELTA = 0, 1
RSD_RADIAL = 3          # rsd_axis value: radial RSD about an observer at the box centre
# get_field ids of the adjoint's cotangents (valid after a gradient evaluation)
FIELD_DRHO = 18         # d logL / d rho
FIELD_DPSI = 19         # d logL / d Psi_j is FIELD_DPSI + j
# bits of the per-chain non-finite flags
NF_STATE, NF_LOGL, NF_GRAD, NF_HAMILTONIAN = 1, 2, 4, 8
W_NONFINITE = 1         # status of fzw_check_finite when some chain is flagged
PLAN_CHECKPOINT = 1     # fzw_plan_create_ex flag: recompute phi_ij in the adjoint
KERNEL_CLASSES = ("z_r2c", "z_c2r", "y_mix", "x_mix", "y_pure", "x_pure", "lpt_fwd", "lpt_bwd", "cic_deposit",
                  "cic_adjoint", "voxel_fwd", "likelihood", "voxel_bwd", "y_mix_multi", "x_mix_multi")
# classes that are one kernel (template) each; the CIC deposit is a sequence
SINGLE_KERNEL_CLASSES = tuple(c for c in KERNEL_CLASSES if c != "cic_deposit")


class FzwError(RuntimeError):
    pass


class CCosmo(ctypes.Structure):
    _fields_ = [("omega_m", ctypes.c_double), ("h", ctypes.c_double), ("sigma8", ctypes.c_double),
                ("n_s", ctypes.c_double), ("d1", ctypes.c_double), ("f_growth", ctypes.c_double),
                ("r_s", ctypes.c_double), ("rsd_axis", ctypes.c_int), ("tau_sc", ctypes.c_double),
                ("x_floor", ctypes.c_double)]


class CWeb(ctypes.Structure):
    _fields_ = [("n_webs", ctypes.c_int), ("kind", ctypes.c_int * 2), ("smooth_r", ctypes.c_double * 2),
                ("ell", ctypes.c_double * 2), ("steepness", ctypes.c_double), ("lambda_th", ctypes.c_double)]


class CDualAvg(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("target", ctypes.c_double), ("gamma", ctypes.c_double),
                ("t0", ctypes.c_double), ("kappa", ctypes.c_double), ("h_bar", ctypes.c_double),
                ("log_eps_bar", ctypes.c_double), ("t", ctypes.c_longlong)]


NUTS_MAX_DEPTH = 12


def nuts_n_uniforms(max_depth: int) -> int:
    """Uniform draws one NUTS transition consumes per chain."""
    return 2 * max_depth + (1 << max_depth) - 1


def load_library(path: str = _LIB_PATH):
    """Load libfzw.so and declare its signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FzwError("libfzw.so is not built at %s; run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    lib.fzw_plan_create.argtypes = [ctypes.POINTER(vp), i, ctypes.POINTER(i), ctypes.POINTER(d),
                                    ctypes.POINTER(CCosmo), ctypes.POINTER(CWeb), vp]
    lib.fzw_plan_create_ex.argtypes = [ctypes.POINTER(vp), i, ctypes.POINTER(i), ctypes.POINTER(d),
                                       ctypes.POINTER(CCosmo), ctypes.POINTER(CWeb), vp, ctypes.c_uint]
    lib.fzw_plan_create_ex.restype = ctypes.c_int
    lib.fzw_plan_destroy.argtypes = [vp]
    lib.fzw_plan_destroy.restype = None
    lib.fzw_set_counts.argtypes = [vp, i, vp]
    lib.fzw_forward.argtypes = [vp, vp, vp, vp, vp]
    lib.fzw_value_and_grad.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.fzw_set_sampling.argtypes = [vp, ctypes.POINTER(i), i, ctypes.POINTER(d), ctypes.POINTER(d)]
    lib.fzw_leapfrog.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, i, vp, vp]
    lib.fzw_get_field.argtypes = [vp, i, i, vp]
    lib.fzw_nonfinite_flags.argtypes = [vp, vp]
    lib.fzw_nonfinite_flags.restype = ctypes.c_int
    lib.fzw_check_finite.argtypes = [vp, ctypes.POINTER(i)]
    lib.fzw_check_finite.restype = ctypes.c_int
    lib.fzw_fft_r2c.argtypes = [vp, i, i, vp, vp]
    lib.fzw_fft_c2r.argtypes = [vp, i, i, vp, vp]
    lib.fzw_set_cic_method.argtypes = [vp, i]
    lib.fzw_set_cic_method.restype = ctypes.c_int
    lib.fzw_timing_enable.argtypes = [vp, i]
    lib.fzw_timing_enable.restype = ctypes.c_int
    lib.fzw_timing_read.argtypes = [vp, i, ctypes.POINTER(d), ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(d)]
    lib.fzw_timing_read.restype = ctypes.c_int
    lib.fzw_fft_schedule.argtypes = [i, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(d)]
    lib.fzw_fft_schedule.restype = ctypes.c_int
    lib.fzw_set_fft_schedule.argtypes = [i, i, i, i]
    lib.fzw_set_fft_schedule.restype = ctypes.c_int
    lib.fzw_chain_offset.argtypes = [vp, i]
    lib.fzw_chain_offset.restype = sz
    lib.fzw_n_regions.argtypes = [vp]
    lib.fzw_workspace_bytes.argtypes = [vp]
    lib.fzw_workspace_bytes.restype = sz
    lib.fzw_last_error.restype = ctypes.c_char_p
    lib.fzw_nuts.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i, vp, vp, vp]
    ll = ctypes.c_longlong
    lib.fzw_welford.argtypes = [vp, vp, vp, vp, ll, i]
    lib.fzw_wiener_start.argtypes = [vp, vp]
    lib.fzw_set_integrator.argtypes = [vp, i]
    lib.fzw_set_sampling_signs.argtypes = [vp, ctypes.POINTER(i), i]
    lib.fzw_power_multipoles.argtypes = [vp, i, vp, vp, d, d, i, vp]
    lib.fzw_bispectrum.argtypes = [vp, i, vp, d, d, d, i, ctypes.POINTER(d), vp]
    lib.fzw_power_multipoles_noalloc.argtypes = [vp, i, vp, vp, d, d, i, vp]
    lib.fzw_power_multipoles_noalloc.restype = ctypes.c_int
    lib.fzw_inverse_mass.argtypes = [vp, vp, vp, ll, i]
    lib.fzw_dual_avg_init.argtypes = [ctypes.POINTER(CDualAvg), d, d]
    lib.fzw_dual_avg_init.restype = None
    lib.fzw_dual_avg_update.argtypes = [ctypes.POINTER(CDualAvg), d]
    lib.fzw_dual_avg_update.restype = d
    lib.fzw_dual_avg_final.argtypes = [ctypes.POINTER(CDualAvg)]
    lib.fzw_dual_avg_final.restype = d
    for name in ("fzw_plan_create", "fzw_set_counts", "fzw_forward", "fzw_value_and_grad",
                 "fzw_set_sampling", "fzw_leapfrog", "fzw_get_field", "fzw_fft_r2c", "fzw_fft_c2r",
                 "fzw_nuts", "fzw_welford", "fzw_inverse_mass", "fzw_wiener_start", "fzw_power_multipoles",
                 "fzw_bispectrum", "fzw_set_integrator", "fzw_set_sampling_signs"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != 0:
        msg = _lib.fzw_last_error().decode() if _lib is not None else ""
        raise FzwError("%s failed with status %d: %s" % (what, status, msg))


def _ptr(t: Optional[torch.Tensor], dtype=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise FzwError("tensor must live on the GPU")
    if dtype is not None and t.dtype != dtype:
        raise FzwError("expected %s, got %s" % (dtype, t.dtype))
    if not t.is_contiguous():
        raise FzwError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class CosmoParams:
    omega_m: float = 0.31
    h: float = 0.68
    sigma8: float = 0.81
    n_s: float = 0.96
    d1: float = 1.0
    f_growth: float = 0.31 ** 0.55
    r_s: float = 4.0
    rsd_axis: int = -1
    tau_sc: float = 0.0
    x_floor: float = 1e-6

    def c(self) -> CCosmo:
        return CCosmo(self.omega_m, self.h, self.sigma8, self.n_s, self.d1, self.f_growth, self.r_s,
                      self.rsd_axis, self.tau_sc, self.x_floor)


@dataclass
class WebParams:
    kinds: Sequence[int] = (WEB_PHI,)
    smooth_r: Sequence[float] = (0.0,)
    ell: Sequence[float] = (0.0,)
    steepness: float = 20.0
    lambda_th: float = 0.1

    def c(self) -> CWeb:
        n = len(self.kinds)
        w = CWeb()
        w.n_webs = n
        for k in range(n):
            w.kind[k] = int(self.kinds[k])
            w.smooth_r[k] = float(self.smooth_r[k])
            w.ell[k] = float(self.ell[k])
        w.steepness = self.steepness
        w.lambda_th = self.lambda_th
        return w


class Plan:
    """A set of chains (meshes) sharing cosmology and web settings."""

    def __init__(self, mesh_n: Sequence[int], box_l: Sequence[float], cosmo: CosmoParams, web: WebParams,
                 device: int = 0, checkpoint: bool = False):
        """checkpoint: keep no first-order Hessian between the forward model and
        the adjoint (recomputed from nu; FZW_PLAN_CHECKPOINT)."""
        lib = load_library()
        self.device = torch.device("cuda", device)
        self.mesh_n = [int(n) for n in mesh_n]
        self.box_l = [float(b) for b in box_l]
        self.n_chains = len(self.mesh_n)
        self.cosmo, self.web = cosmo, web
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            arr_n = (ctypes.c_int * self.n_chains)(*self.mesh_n)
            arr_l = (ctypes.c_double * self.n_chains)(*self.box_l)
            cc, cw = cosmo.c(), web.c()
            _check(lib.fzw_plan_create_ex(ctypes.byref(h), self.n_chains, arr_n, arr_l, ctypes.byref(cc),
                                          ctypes.byref(cw), ctypes.c_void_p(self.stream.cuda_stream),
                                          PLAN_CHECKPOINT if checkpoint else 0), "fzw_plan_create")
        self._h = h
        self.n_regions = lib.fzw_n_regions(h)
        self.offsets = [int(lib.fzw_chain_offset(h, c)) for c in range(self.n_chains)]
        self.total_voxels = self.offsets[-1] + self.mesh_n[-1] ** 3
        self.nfree = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.fzw_plan_destroy(h)
            self._h = None

    @property
    def workspace_bytes(self) -> int:
        return int(_lib.fzw_workspace_bytes(self._h))

    def chain_view(self, packed: torch.Tensor, c: int) -> torch.Tensor:
        n = self.mesh_n[c]
        o = self.offsets[c]
        return packed[o:o + n ** 3].view(n, n, n)

    def set_counts(self, chain: int, counts: torch.Tensor):
        """counts: uint16 data on the GPU (any int16/uint16 tensor with N^3 entries)."""
        if counts.dtype not in (torch.int16, torch.uint16):
            raise FzwError("counts must be 16-bit")
        _check(_lib.fzw_set_counts(self._h, chain, _ptr(counts.contiguous())), "fzw_set_counts")

    def forward(self, nu: torch.Tensor, bias: torch.Tensor, want_nbar: bool = False):
        logl = torch.empty(self.n_chains, dtype=torch.float64, device=self.device)
        nbar = torch.empty_like(nu) if want_nbar else None
        _check(_lib.fzw_forward(self._h, _ptr(nu, torch.float32), _ptr(bias, torch.float32), _ptr(nbar),
                                _ptr(logl)), "fzw_forward")
        return (logl, nbar) if want_nbar else logl

    def value_and_grad(self, nu: torch.Tensor, bias: torch.Tensor, out=None):
        if out is None:
            out = (torch.empty(self.n_chains, dtype=torch.float64, device=self.device),
                   torch.empty_like(nu), torch.empty_like(bias))
        logl, dnu, dbias = out
        _check(_lib.fzw_value_and_grad(self._h, _ptr(nu, torch.float32), _ptr(bias, torch.float32),
                                       _ptr(logl, torch.float64), _ptr(dnu, torch.float32),
                                       _ptr(dbias, torch.float32)), "fzw_value_and_grad")
        return logl, dnu, dbias

    def set_sampling(self, tie: Sequence[int], mu: Sequence[float], sigma: Sequence[float]):
        nf = len(mu)
        arr_t = (ctypes.c_int * len(tie))(*[int(x) for x in tie])
        arr_m = (ctypes.c_double * max(nf, 1))(*[float(x) for x in mu])
        arr_s = (ctypes.c_double * max(nf, 1))(*[float(x) for x in sigma])
        _check(_lib.fzw_set_sampling(self._h, arr_t, nf, arr_m, arr_s), "fzw_set_sampling")
        self.nfree = nf

    def set_sampling_signs(self, signs: Sequence[int]):
        """Free parameter f is signs[f] * exp(u_f) (after set_sampling)."""
        arr = (ctypes.c_int * max(len(signs), 1))(*[int(x) for x in signs])
        _check(_lib.fzw_set_sampling_signs(self._h, arr, len(signs)), "fzw_set_sampling_signs")

    def leapfrog(self, nu, u, p_nu, p_u, bias_base, minv_nu, minv_u, step, n_steps, h_start=None, h_end=None):
        if h_start is None:
            h_start = torch.empty(self.n_chains, dtype=torch.float64, device=self.device)
        if h_end is None:
            h_end = torch.empty(self.n_chains, dtype=torch.float64, device=self.device)
        _check(_lib.fzw_leapfrog(self._h, _ptr(nu, torch.float32), _ptr(u), _ptr(p_nu, torch.float32), _ptr(p_u),
                                 _ptr(bias_base, torch.float32), _ptr(minv_nu, torch.float32), _ptr(minv_u),
                                 _ptr(step, torch.float32), int(n_steps), _ptr(h_start, torch.float64),
                                 _ptr(h_end, torch.float64)), "fzw_leapfrog")
        return h_start, h_end

    def nuts(self, nu, u, z_nu, z_u, bias_base, minv_nu, minv_u, step, uniforms, max_depth):
        """One no-U-turn transition per chain (fzw_nuts); nu and u are replaced
        by the new state.  Returns (potential, accept_stat, stats[chains][3])."""
        pot = torch.empty(self.n_chains, dtype=torch.float64, device=self.device)
        acc = torch.empty(self.n_chains, dtype=torch.float64, device=self.device)
        stats = torch.empty((self.n_chains, 3), dtype=torch.int32, device=self.device)
        if uniforms.shape[-1] != nuts_n_uniforms(max_depth) or not uniforms.is_contiguous():
            raise FzwError("uniforms must be contiguous [chains][%d]" % nuts_n_uniforms(max_depth))
        _check(_lib.fzw_nuts(self._h, _ptr(nu, torch.float32), _ptr(u), _ptr(z_nu, torch.float32), _ptr(z_u),
                             _ptr(bias_base, torch.float32), _ptr(minv_nu, torch.float32), _ptr(minv_u),
                             _ptr(step, torch.float32), _ptr(uniforms, torch.float32), int(max_depth),
                             _ptr(pot, torch.float64), _ptr(acc, torch.float64), _ptr(stats, torch.int32)),
               "fzw_nuts")
        return pot, acc, stats

    def wiener_start(self, nu=None):
        """White-noise start of every chain from its Wiener-filtered counts
        (fzw_wiener_start); returns the packed field."""
        if nu is None:
            nu = torch.empty(self.total_voxels, dtype=torch.float32, device=self.device)
        _check(_lib.fzw_wiener_start(self._h, _ptr(nu, torch.float32)), "fzw_wiener_start")
        return nu

    def power_multipoles(self, a, b=None, k_lo=0.0, dk=None, nbins=32, mesh_n=None):
        """Monopole and quadrupole of the auto or cross spectrum of fields on
        one of the plan's meshes: tensor [nbins][4] = (k, modes, P0, P2)."""
        n = mesh_n or round(a.numel() ** (1.0 / 3.0))
        out = torch.empty((nbins, 4), dtype=torch.float64, device=self.device)
        _check(_lib.fzw_power_multipoles(self._h, int(n), _ptr(a, torch.float32), _ptr(b, torch.float32),
                                         float(k_lo), float(dk), int(nbins), _ptr(out, torch.float64)),
               "fzw_power_multipoles")
        return out

    def power_multipoles_noalloc(self, a, b=None, k_lo=0.0, dk=None, nbins=32, mesh_n=None, out=None):
        """power_multipoles through the library's allocation-free entry point
        (its partials live in a fixed device array); `out` may be passed so
        that nothing is allocated on this side either."""
        n = mesh_n or round(a.numel() ** (1.0 / 3.0))
        if out is None:
            out = torch.empty((nbins, 4), dtype=torch.float64, device=self.device)
        _check(_lib.fzw_power_multipoles_noalloc(self._h, int(n), _ptr(a, torch.float32), _ptr(b, torch.float32),
                                                 float(k_lo), float(dk), int(nbins), _ptr(out, torch.float64)),
               "fzw_power_multipoles_noalloc")
        return out

    def bispectrum(self, delta, k1, k2, dk, thetas, mesh_n=None):
        """(k3, B, Q, triangles) per opening angle: tensor [len(thetas)][4]."""
        n = mesh_n or round(delta.numel() ** (1.0 / 3.0))
        th = (ctypes.c_double * len(thetas))(*[float(t) for t in thetas])
        out = torch.empty((len(thetas), 4), dtype=torch.float64, device=self.device)
        _check(_lib.fzw_bispectrum(self._h, int(n), _ptr(delta, torch.float32), float(k1), float(k2), float(dk),
                                   len(thetas), th, _ptr(out, torch.float64)), "fzw_bispectrum")
        return out

    def welford(self, x, mean, m2, count):
        """Adds sample `count` (1-based) x to the running mean and m2."""
        _check(_lib.fzw_welford(self._h, _ptr(x, torch.float32), _ptr(mean, torch.float32), _ptr(m2, torch.float32),
                                x.numel(), int(count)), "fzw_welford")

    def inverse_mass(self, m2, minv, count):
        _check(_lib.fzw_inverse_mass(self._h, _ptr(m2, torch.float32), _ptr(minv, torch.float32), m2.numel(),
                                     int(count)), "fzw_inverse_mass")

    INTEGRATORS = {"leapfrog": 0, "blanes2": 1, "yoshida4": 2}

    def set_integrator(self, scheme: str):
        """Splitting scheme of `leapfrog` trajectories: 'leapfrog' (default),
        'blanes2' (two-stage, two gradients per step) or 'yoshida4' (fourth
        order, three gradients per step)."""
        _check(_lib.fzw_set_integrator(self._h, self.INTEGRATORS[scheme]), "fzw_set_integrator")

    def set_cic_method(self, method: str):
        """'sorted' (counting sort + gather, default) or 'atomic' (fixed-point
        integer atomics); both give bit-identical densities."""
        _check(_lib.fzw_set_cic_method(self._h, {"sorted": 0, "atomic": 1}[method]), "fzw_set_cic_method")

    def timing(self, on: bool):
        """Bracket every later launch with HIP events (per kernel class)."""
        _check(_lib.fzw_timing_enable(self._h, 1 if on else 0), "fzw_timing_enable")

    def timing_report(self):
        """{class: (total_ms, launches, algorithmic_bytes)} since timing(True)."""
        out = {}
        for k, name in enumerate(KERNEL_CLASSES):
            ms, n, b = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
            _check(_lib.fzw_timing_read(self._h, k, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)),
                   "fzw_timing_read")
            out[name] = (ms.value, n.value, b.value)
        return out

    def nonfinite_flags(self) -> torch.Tensor:
        """Per-chain non-finite flags (NF_* bits) of the last evaluation call,
        as an int32 device tensor (copied on the plan's stream)."""
        out = torch.empty(self.n_chains, dtype=torch.int32, device=self.device)
        _check(_lib.fzw_nonfinite_flags(self._h, _ptr(out, torch.int32)), "fzw_nonfinite_flags")
        return out

    def check_finite(self):
        """(all finite, per-chain flags): synchronises the plan's stream."""
        arr = (ctypes.c_int * self.n_chains)()
        st = _lib.fzw_check_finite(self._h, arr)
        if st < 0:
            _check(st, "fzw_check_finite")
        return st == 0, [int(x) for x in arr]

    def get_field(self, chain: int, field_id: int) -> torch.Tensor:
        n = self.mesh_n[chain]
        out = torch.empty((n, n, n), dtype=torch.float32, device=self.device)
        _check(_lib.fzw_get_field(self._h, chain, field_id, _ptr(out)), "fzw_get_field")
        return out

    def fft_r2c(self, x: torch.Tensor) -> torch.Tensor:
        n = x.shape[-1]
        b = x.numel() // n ** 3
        out = torch.empty((b, n, n, n // 2 + 1), dtype=torch.complex64, device=self.device)
        _check(_lib.fzw_fft_r2c(self._h, n, b, _ptr(x.contiguous(), torch.float32), _ptr(out)), "fzw_fft_r2c")
        return out

    def fft_c2r(self, x: torch.Tensor) -> torch.Tensor:
        n = x.shape[-2]
        b = x.numel() // (n * n * (n // 2 + 1))
        out = torch.empty((b, n, n, n), dtype=torch.float32, device=self.device)
        _check(_lib.fzw_fft_c2r(self._h, n, b, _ptr(x.contiguous(), torch.complex64), _ptr(out)), "fzw_fft_c2r")
        return out


FFT_FAMILIES = ("four-step", "stockham")


class DualAveraging:
    """Step-size adaptation by dual averaging (fzw_dual_avg_*), one per chain."""

    def __init__(self, eps0: float, target: float = 0.8):
        load_library()
        self._s = CDualAvg()
        _lib.fzw_dual_avg_init(ctypes.byref(self._s), float(eps0), float(target))

    def update(self, accept_stat: float) -> float:
        return _lib.fzw_dual_avg_update(ctypes.byref(self._s), float(accept_stat))

    def final(self) -> float:
        return _lib.fzw_dual_avg_final(ctypes.byref(self._s))


def fft_schedule(mesh_n: int):
    """The FFT kernel schedule the library picked for a mesh size (after a
    plan of that size exists): {'z', 'xy', 'pure'} -> (family, us four-step,
    us alternative)."""
    lib = load_library()
    z, xy, pure = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    us = (ctypes.c_double * 6)()
    _check(lib.fzw_fft_schedule(int(mesh_n), ctypes.byref(z), ctypes.byref(xy), ctypes.byref(pure), us),
           "fzw_fft_schedule")
    alt = {"z": "stockham", "xy": "stockham", "pure": "mixing"}
    out = {}
    for k, (name, v) in enumerate((("z", z.value), ("xy", xy.value), ("pure", pure.value))):
        fam = "four-step" if v == 0 else alt[name]
        out[name] = (fam, us[2 * k], us[2 * k + 1])
    return out


def set_fft_schedule(mesh_n: int, z: str = "four-step", xy: str = "four-step", pure: str = "four-step"):
    """Force the FFT kernel families of a mesh size ('four-step' or the
    alternative: 'stockham' for z and xy, 'mixing' for pure)."""
    code = {"four-step": 0, "stockham": 1, "mixing": 1}
    _check(load_library().fzw_set_fft_schedule(int(mesh_n), code[z], code[xy], code[pure]),
           "fzw_set_fft_schedule")


class LogLikelihood(torch.autograd.Function):
    """logL(nu, bias) per chain with the library's hand-written adjoint as backward."""

    @staticmethod
    def forward(ctx, nu, bias, plan: Plan):
        logl, dnu, dbias = plan.value_and_grad(nu.detach().contiguous(), bias.detach().contiguous())
        ctx.save_for_backward(dnu, dbias)
        ctx.plan = plan
        return logl

    @staticmethod
    def backward(ctx, g):
        # chains are packed back to back whatever the shape of nu (flat, or
        # [chains][N][N][N] when every chain has the same mesh): scale chain c's
        # slice of the flat gradient by g[c]
        dnu, dbias = ctx.saved_tensors
        plan = ctx.plan
        flat = dnu.reshape(-1)
        gn = torch.empty_like(flat)
        for c in range(plan.n_chains):
            o, n = plan.offsets[c], plan.mesh_n[c] ** 3
            gn[o:o + n] = flat[o:o + n] * g[c].to(dnu.dtype)
        gb = (dbias.reshape(plan.n_chains, -1) * g.to(dbias.dtype).view(-1, 1)).view_as(dbias)
        return gn.view_as(dnu), gb, None
