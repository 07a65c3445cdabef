"""Thin ctypes binding of libletkf (include/letkf.h): argument marshalling only.

Every step of the frame runs in the HIP library; torch is used for device
memory and streams.  Importing this module loads the library and raises when
it is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref
from dataclasses import dataclass

import numpy as np
# torch first: its bundled HIP runtime (soname libamdhip64.so.7) is then the one
# libletkf binds to, so the process holds a single HIP runtime and torch's
# device buffers and streams are valid in the library.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
# LETKF_LIBRARY selects another build of the same ABI (e.g. an instrumented one).
LIB_PATH = os.environ.get("LETKF_LIBRARY", os.path.join(_HERE, "libletkf.so"))

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
lib = C.CDLL(LIB_PATH)

OK, E_INVAL, E_NOMEM, E_DEVICE, E_NONFINITE, E_NOCONV, E_STATE = 0, -1, -2, -3, -4, -5, -6
FP32, FP64 = 0, 1
FLAG_NONFINITE, FLAG_NOCONV = 1, 2
TRANSFORM_NS64, TRANSFORM_NS32, TRANSFORM_EVD, TRANSFORM_NSP, TRANSFORM_NSP_MIXED = 0, 1, 2, 3, 4
MODEL_PHASE, MODEL_CLOSED_LOOP = 0, 1
GATHER_CONCAT, GATHER_BLEND = 0, 1
LOCALISATION_DOMAIN, LOCALISATION_COVARIANCE = 0, 1
ORDER_ROW, ORDER_XCD, ORDER_XCD_PAIRED = 0, 1, 2


class Config(C.Structure):
    _fields_ = [
        ("n_sub", C.c_int32),
        ("subap_mask", C.POINTER(C.c_uint8)),
        ("obscuration", C.c_double),
        ("m", C.c_int32),
        ("domain_size", C.c_int32),
        ("halo", C.c_int32),
        ("rho", C.c_double),
        ("r_diag", C.POINTER(C.c_double)),
        ("r_sigma2", C.c_double),
        ("r_scale", C.c_double),
        ("ar_coeff", C.c_double),
        ("taper_c", C.c_double),
        ("noise_bank", C.POINTER(C.c_float)),
        ("bank_screens", C.c_int32),
        ("bank_side", C.c_int32),
        ("seed", C.c_uint64),
        ("precision", C.c_int32),
        ("jacobi_tol", C.c_double),
        ("max_sweeps", C.c_int32),
        ("piston_removal", C.c_int32),
        ("transform", C.c_int32),
        ("model", C.c_int32),
        ("ar2_coeff", C.c_double),
        ("refit_forgetting", C.c_double),
        ("gather_mode", C.c_int32),
        ("localisation", C.c_int32),
    ]


class Sizes(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int64),
        ("n_slopes", C.c_int64),
        ("n_domains", C.c_int64),
        ("ensemble_elems", C.c_int64),
        ("obs_total", C.c_int64),
        ("m", C.c_int32),
        ("max_owned", C.c_int32),
        ("max_obs", C.c_int32),
        ("max_patch", C.c_int32),
        ("n_sub", C.c_int32),
        ("n_instances", C.c_int32),
    ]


_P = C.c_void_p
_I32P = C.POINTER(C.c_int32)
_SIGS = {
    "letkf_create": (C.c_int, [C.POINTER(Config), C.c_int32, C.c_int32, C.POINTER(_P)]),
    "letkf_destroy": (None, [_P]),
    "letkf_strerror": (C.c_char_p, [C.c_int]),
    "letkf_last_error": (C.c_char_p, []),
    "letkf_query": (C.c_int, [_P, C.c_int32, C.POINTER(Sizes)]),
    "letkf_plan": (C.c_int, [C.POINTER(Config), C.POINTER(Sizes), _I32P, _I32P, _I32P, _I32P, _I32P, _I32P]),
    "letkf_geometry": (C.c_int, [_P, C.c_int32, _I32P, _I32P, _I32P, _I32P, _I32P, _I32P]),
    "letkf_forecast": (C.c_int, [_P, _P, _P]),
    "letkf_analyse": (C.c_int, [_P, _P, _P]),
    "letkf_step": (C.c_int, [_P, _P, _P, _P]),
    "letkf_step_plain": (C.c_int, [_P, _P, _P, _P]),
    "letkf_get_ensemble": (C.c_int, [_P, _P, C.c_int]),
    "letkf_set_ensemble": (C.c_int, [_P, _P, C.c_int]),
    "letkf_get_forecast": (C.c_int, [_P, _P, C.c_int]),
    "letkf_get_mean": (C.c_int, [_P, _P, C.c_int]),
    "letkf_get_command": (C.c_int, [_P, _P, C.c_int]),
    "letkf_set_command": (C.c_int, [_P, _P, _P, C.c_int]),
    "letkf_get_model": (C.c_int, [_P, _P, _P]),
    "letkf_reset_refit": (C.c_int, [_P]),
    "letkf_get_frame": (C.c_int, [_P, C.POINTER(C.c_uint32)]),
    "letkf_set_frame": (C.c_int, [_P, C.c_uint32]),
    "letkf_status": (C.c_int, [_P, _I32P]),
    "letkf_set_params": (C.c_int, [_P, C.c_int32, C.c_double, C.c_double, C.c_double]),
    "letkf_slopes": (C.c_int, [_P, _P, _P, _P]),
    "letkf_set_schedule": (C.c_int, [_P, C.c_int32, C.c_int32]),
    "letkf_get_schedule": (C.c_int, [_P, _I32P, _I32P]),
    "letkf_autotune": (C.c_int, [_P, _P, _P, C.c_int32, C.c_char_p, _P]),
    "letkf_eigh_spd": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_double, C.c_int32, _P, _P, _P, _P]),
    "letkf_residual_variance": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "letkf_residual_variance_adjoint": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "letkf_adjoint": (C.c_int, [_P, _P, _P, C.c_uint32, _P, _P, _P, _P]),
    "letkf_adjoint_noalloc": (C.c_int, [_P, _P, _P, C.c_uint32, _P, _P, _P, _P]),
    "letkf_set_timing": (C.c_int, [_P, C.c_int32]),
    "letkf_analysis_times": (C.c_int, [_P, C.POINTER(C.c_float), C.c_int32, _I32P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class LetkfError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = lib.letkf_strerror(code).decode()
        detail = lib.letkf_last_error().decode()
        super().__init__(f"{where}: {msg} ({code}){': ' + detail if detail else ''}")


def _check(code: int, where: str) -> int:
    if code != OK:
        raise LetkfError(code, where)
    return code


@dataclass
class InstanceSpec:
    """One adaptive-optics instance (mirrors letkf_config)."""
    n_sub: int
    m: int
    domain_size: int = 4
    halo: int = 1
    obscuration: float = 0.0
    mask: np.ndarray | None = None        # (N, N) bool; None = annulus rule
    rho: float = 1.05
    r_diag: np.ndarray | None = None      # (p,) float64; None = r_sigma2
    r_sigma2: float = 0.01
    r_scale: float = 1.0
    ar_coeff: float = 0.99
    taper_c: float = 0.0
    noise_bank: np.ndarray | None = None  # (screens, side, side) float32
    seed: int = 0
    precision: int = FP32
    jacobi_tol: float = 0.0
    max_sweeps: int = 0
    piston: bool = False                  # differential-piston removal after the gather
    transform: int = TRANSFORM_NSP_MIXED  # how W, w come from A~ (NSP_MIXED, NSP, NS64, NS32 or the Jacobi EVD)
    model: int = MODEL_PHASE              # delay-free phase state, or the closed AO loop (Sec. 2.2)
    ar2_coeff: float = 0.0                # a2 of an AR(2) turbulence model (0: AR(1))
    refit_forgetting: float = 0.0         # online AR(1) refit with this forgetting factor (0: off)
    gather_mode: int = 0                  # GATHER_CONCAT, or GATHER_BLEND (aligned, tent-weighted patches)
    localisation: int = 0                 # LOCALISATION_DOMAIN, or LOCALISATION_COVARIANCE (Schur-tapered P)


def _config(spec: InstanceSpec, keep: list) -> Config:
    c = Config()
    c.n_sub = spec.n_sub
    if spec.mask is not None:
        mk = np.ascontiguousarray(np.asarray(spec.mask, dtype=np.uint8))
        keep.append(mk)
        c.subap_mask = mk.ctypes.data_as(C.POINTER(C.c_uint8))
    c.obscuration = spec.obscuration
    c.m = spec.m
    c.domain_size = spec.domain_size
    c.halo = spec.halo
    c.rho = spec.rho
    if spec.r_diag is not None:
        r = np.ascontiguousarray(np.asarray(spec.r_diag, dtype=np.float64))
        keep.append(r)
        c.r_diag = r.ctypes.data_as(C.POINTER(C.c_double))
    c.r_sigma2 = spec.r_sigma2
    c.r_scale = spec.r_scale
    c.ar_coeff = spec.ar_coeff
    c.taper_c = spec.taper_c
    if spec.noise_bank is not None:
        b = np.ascontiguousarray(np.asarray(spec.noise_bank, dtype=np.float32))
        keep.append(b)
        c.noise_bank = b.ctypes.data_as(C.POINTER(C.c_float))
        c.bank_screens = b.shape[0]
        c.bank_side = b.shape[1]
    c.seed = spec.seed
    c.precision = spec.precision
    c.jacobi_tol = spec.jacobi_tol
    c.max_sweeps = spec.max_sweeps
    c.piston_removal = 1 if spec.piston else 0
    c.transform = spec.transform
    c.model = spec.model
    c.ar2_coeff = spec.ar2_coeff
    c.refit_forgetting = spec.refit_forgetting
    c.gather_mode = spec.gather_mode
    c.localisation = spec.localisation
    return c


def _maps(call, n_nodes: int, n_domains: int, obs_total: int):
    node_ij = np.zeros(2 * n_nodes, dtype=np.int32)
    owner = np.zeros(n_nodes, dtype=np.int32)
    obs_off = np.zeros(n_domains + 1, dtype=np.int32)
    obs_idx = np.zeros(max(obs_total, 1), dtype=np.int32)
    own_off = np.zeros(n_domains + 1, dtype=np.int32)
    own_idx = np.zeros(max(n_nodes, 1), dtype=np.int32)
    ptr = lambda a: a.ctypes.data_as(_I32P)
    call(ptr(node_ij), ptr(owner), ptr(obs_off), ptr(obs_idx), ptr(own_off), ptr(own_idx))
    return {"node_ij": node_ij.reshape(-1, 2), "owner": owner, "obs_off": obs_off,
            "obs_idx": obs_idx[:obs_total], "own_off": own_off, "own_idx": own_idx[:n_nodes]}


def plan(spec: InstanceSpec) -> tuple[dict, dict]:
    """Host-only planning (letkf_plan): sizes and integer maps, no device."""
    keep: list = []
    cfg = _config(spec, keep)
    s = Sizes()
    _check(lib.letkf_plan(C.byref(cfg), C.byref(s), None, None, None, None, None, None), "letkf_plan")
    sizes = {f: getattr(s, f) for f, _ in Sizes._fields_}
    maps = _maps(lambda *a: _check(lib.letkf_plan(C.byref(cfg), None, *a), "letkf_plan"),
                 s.n_nodes, s.n_domains, s.obs_total)
    return sizes, maps


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Letkf:
    """A handle over one or more instances (letkf_create ... letkf_destroy)."""

    def __init__(self, specs, device: int = 0):
        specs = list(specs) if isinstance(specs, (list, tuple)) else [specs]
        keep: list = []
        arr = (Config * len(specs))(*[_config(s, keep) for s in specs])
        h = C.c_void_p()
        _check(lib.letkf_create(arr, len(specs), device, C.byref(h)), "letkf_create")
        self._h = h
        # the destroy function is bound now, so that a handle still alive at
        # interpreter exit is destroyed even after the module globals are gone
        self._fin = weakref.finalize(self, lib.letkf_destroy, h)
        self.device = device
        self.specs = specs
        self.fp64 = specs[0].precision == FP64
        self.sizes = self.query(-1)
        self.inst_sizes = [self.query(i) for i in range(len(specs))]

    def close(self):
        fin = getattr(self, "_fin", None)
        if fin is not None:
            fin()          # letkf_destroy, at most once
        self._h = None

    # -- sizes and maps
    def query(self, instance: int = -1) -> dict:
        s = Sizes()
        _check(lib.letkf_query(self._h, instance, C.byref(s)), "letkf_query")
        return {f: getattr(s, f) for f, _ in Sizes._fields_}

    def geometry(self, instance: int) -> dict:
        s = self.inst_sizes[instance]
        return _maps(lambda *a: _check(lib.letkf_geometry(self._h, instance, *a), "letkf_geometry"),
                     s["n_nodes"], s["n_domains"], s["obs_total"])

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.fp64 else torch.float32

    def _check_tensor(self, t, n, name):
        if t is None:
            return
        if not t.is_cuda or t.dtype != self.dtype or not t.is_contiguous() or t.numel() < n:
            raise ValueError(f"{name}: need a contiguous {self.dtype} device tensor of >= {n} elements")

    # -- frame
    def forecast(self, V=None, stream=None):
        self._check_tensor(V, self.sizes["ensemble_elems"], "V")
        _check(lib.letkf_forecast(self._h, _ptr(V), _stream(stream)), "letkf_forecast")

    def analyse(self, y, stream=None):
        self._check_tensor(y, self.sizes["n_slopes"], "y")
        _check(lib.letkf_analyse(self._h, _ptr(y), _stream(stream)), "letkf_analyse")

    def step(self, y, V=None, stream=None):
        self._check_tensor(V, self.sizes["ensemble_elems"], "V")
        self._check_tensor(y, self.sizes["n_slopes"], "y")
        _check(lib.letkf_step(self._h, _ptr(V), _ptr(y), _stream(stream)), "letkf_step")

    def step_plain(self, y, V=None, stream=None):
        self._check_tensor(V, self.sizes["ensemble_elems"], "V")
        self._check_tensor(y, self.sizes["n_slopes"], "y")
        _check(lib.letkf_step_plain(self._h, _ptr(V), _ptr(y), _stream(stream)), "letkf_step_plain")

    # -- state
    def get_ensemble(self):
        import torch
        out = torch.empty(self.sizes["ensemble_elems"], dtype=self.dtype, device=f"cuda:{self.device}")
        _check(lib.letkf_get_ensemble(self._h, _ptr(out), 1), "letkf_get_ensemble")
        return out

    def set_ensemble(self, x):
        self._check_tensor(x, self.sizes["ensemble_elems"], "x")
        _check(lib.letkf_set_ensemble(self._h, _ptr(x), 1), "letkf_set_ensemble")

    def get_forecast(self):
        import torch
        out = torch.empty(self.sizes["ensemble_elems"], dtype=self.dtype, device=f"cuda:{self.device}")
        _check(lib.letkf_get_forecast(self._h, _ptr(out), 1), "letkf_get_forecast")
        return out

    def get_mean(self):
        import torch
        out = torch.empty(self.sizes["n_nodes"], dtype=self.dtype, device=f"cuda:{self.device}")
        _check(lib.letkf_get_mean(self._h, _ptr(out), 1), "letkf_get_mean")
        return out

    def get_command(self):
        """The latest closed-loop command u_k per node (all instances)."""
        import torch
        out = torch.empty(self.sizes["n_nodes"], dtype=self.dtype, device=f"cuda:{self.device}")
        _check(lib.letkf_get_command(self._h, _ptr(out), 1), "letkf_get_command")
        return out

    def set_command(self, u_prev1, u_prev2):
        """Set the command history (u_{k-1}, u_{k-2}), device tensors [n_nodes]."""
        _check(lib.letkf_set_command(self._h, _ptr(u_prev1), _ptr(u_prev2), 1), "letkf_set_command")

    def get_model(self):
        """(a, noise scale) per instance that the next forecast uses."""
        a = np.zeros(len(self.specs), dtype=np.float64)
        v = np.zeros(len(self.specs), dtype=np.float64)
        _check(lib.letkf_get_model(self._h, a.ctypes.data, v.ctypes.data), "letkf_get_model")
        return a, v

    def reset_refit(self):
        """Restart the online refit (sums cleared, a = ar_coeff)."""
        _check(lib.letkf_reset_refit(self._h), "letkf_reset_refit")

    def get_frame(self) -> int:
        f = C.c_uint32()
        _check(lib.letkf_get_frame(self._h, C.byref(f)), "letkf_get_frame")
        return f.value

    def set_frame(self, frame: int):
        _check(lib.letkf_set_frame(self._h, frame), "letkf_set_frame")

    def status(self):
        """(return code, per-domain flags in (instance, domain) order)."""
        f = np.zeros(self.sizes["n_domains"], dtype=np.int32)
        rc = lib.letkf_status(self._h, f.ctypes.data_as(_I32P))
        if rc not in (OK, E_NOCONV, E_NONFINITE):
            _check(rc, "letkf_status")
        return rc, f

    def set_params(self, instance: int, rho: float, r_scale: float, taper_c: float):
        _check(lib.letkf_set_params(self._h, instance, rho, r_scale, taper_c), "letkf_set_params")

    def slopes(self, phase, out=None, stream=None):
        import torch
        self._check_tensor(phase, self.sizes["n_nodes"], "phase")
        if out is None:
            out = torch.empty(self.sizes["n_slopes"], dtype=self.dtype, device=phase.device)
        _check(lib.letkf_slopes(self._h, _ptr(phase), _ptr(out), _stream(stream)), "letkf_slopes")
        return out

    def set_schedule(self, use_graph: bool, order: int):
        """use_graph for letkf_step; order: ORDER_ROW, ORDER_XCD (True) or ORDER_XCD_PAIRED."""
        _check(lib.letkf_set_schedule(self._h, int(use_graph), int(order)), "letkf_set_schedule")

    def get_schedule(self):
        g, x = C.c_int32(), C.c_int32()
        _check(lib.letkf_get_schedule(self._h, C.byref(g), C.byref(x)), "letkf_get_schedule")
        return bool(g.value), int(x.value)

    def autotune(self, y, V=None, frames: int = 20, cache_path: str | None = None, stream=None):
        _check(lib.letkf_autotune(self._h, _ptr(V), _ptr(y), frames,
                                  cache_path.encode() if cache_path else None, _stream(stream)),
               "letkf_autotune")
        return self.get_schedule()

    # -- timing
    def set_timing(self, enable: bool):
        _check(lib.letkf_set_timing(self._h, int(enable)), "letkf_set_timing")

    def analysis_times(self, max_n: int = 100000) -> np.ndarray:
        """Durations (ms) of the analysis launches recorded since set_timing."""
        buf = np.zeros(max_n, dtype=np.float32)
        n = C.c_int32()
        _check(lib.letkf_analysis_times(self._h, buf.ctypes.data_as(C.POINTER(C.c_float)), max_n,
                                        C.byref(n)), "letkf_analysis_times")
        return buf[:min(n.value, max_n)].copy()

    # -- loss and adjoint
    def _check_f64(self, t, n, name):
        import torch
        if t is None:
            return
        if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or t.numel() < n:
            raise ValueError(f"{name}: need a contiguous float64 device tensor of >= {n} elements")

    def residual_variance(self, truth, acc, xa=None, weights=None, stream=None):
        """acc[i] += weights[i] * residual variance of instance i's analysis mean."""
        n = self.sizes["n_instances"]
        self._check_tensor(truth, self.sizes["n_nodes"], "truth")
        self._check_tensor(xa, self.sizes["ensemble_elems"], "xa")
        self._check_f64(acc, n, "acc")
        self._check_f64(weights, n, "weights")
        _check(lib.letkf_residual_variance(self._h, _ptr(xa), _ptr(truth), _ptr(weights), _ptr(acc),
                                           _stream(stream)), "letkf_residual_variance")

    def residual_variance_adjoint(self, truth, xbar, xa=None, weights=None, stream=None):
        """xbar += weights[i] * d(residual variance of instance i) / d X_a."""
        self._check_tensor(truth, self.sizes["n_nodes"], "truth")
        self._check_tensor(xa, self.sizes["ensemble_elems"], "xa")
        self._check_tensor(xbar, self.sizes["ensemble_elems"], "xbar")
        self._check_f64(weights, self.sizes["n_instances"], "weights")
        _check(lib.letkf_residual_variance_adjoint(self._h, _ptr(xa), _ptr(truth), _ptr(weights),
                                                   _ptr(xbar), _stream(stream)),
               "letkf_residual_variance_adjoint")

    def adjoint(self, xa_prev, y, xbar, theta_bar, frame: int, V=None, stream=None):
        """Reverse of one frame (letkf_adjoint): xbar becomes the adjoint of
        xa_prev and theta_bar[3 i:3 i + 3] gains d/d(rho, r_scale, taper_c)."""
        self._check_tensor(xa_prev, self.sizes["ensemble_elems"], "xa_prev")
        self._check_tensor(y, self.sizes["n_slopes"], "y")
        self._check_tensor(xbar, self.sizes["ensemble_elems"], "xbar")
        self._check_tensor(V, self.sizes["ensemble_elems"], "V")
        self._check_f64(theta_bar, 3 * self.sizes["n_instances"], "theta_bar")
        _check(lib.letkf_adjoint(self._h, _ptr(xa_prev), _ptr(V), frame, _ptr(y), _ptr(xbar),
                                 _ptr(theta_bar), _stream(stream)), "letkf_adjoint")

    def adjoint_noalloc(self, xa_prev, y, xbar, theta_bar, frame: int, V=None, stream=None):
        """letkf_adjoint_noalloc: as adjoint, with the library's fixed device
        scratch in place of buffers allocated on first use."""
        self._check_tensor(xa_prev, self.sizes["ensemble_elems"], "xa_prev")
        self._check_tensor(y, self.sizes["n_slopes"], "y")
        self._check_tensor(xbar, self.sizes["ensemble_elems"], "xbar")
        self._check_tensor(V, self.sizes["ensemble_elems"], "V")
        self._check_f64(theta_bar, 3 * self.sizes["n_instances"], "theta_bar")
        _check(lib.letkf_adjoint_noalloc(self._h, _ptr(xa_prev), _ptr(V), frame, _ptr(y), _ptr(xbar),
                                         _ptr(theta_bar), _stream(stream)), "letkf_adjoint_noalloc")


def eigh_spd(A, tol: float = 1e-12, max_sweeps: int = 30, stream=None):
    """letkf_eigh_spd on a (batch, m, m) float64 device tensor of SPD matrices:
    returns (Q, lam, sweeps) with A = Q diag(lam) Q^T (unsorted)."""
    import torch
    if A.dtype != torch.float64 or not A.is_cuda or A.dim() != 3 or A.shape[1] != A.shape[2]:
        raise ValueError("A must be a (batch, m, m) float64 CUDA tensor")
    A = A.contiguous()
    b, m, _ = A.shape
    Q = torch.empty_like(A)
    lam = torch.empty((b, m), dtype=torch.float64, device=A.device)
    sw = torch.empty(b, dtype=torch.int32, device=A.device)
    _check(lib.letkf_eigh_spd(_ptr(A), m, b, tol, max_sweeps, _ptr(Q), _ptr(lam), _ptr(sw),
                              _stream(stream)), "letkf_eigh_spd")
    return Q, lam, sw


def header_symbols(header_path: str) -> list[str]:
    """Function names declared in include/letkf.h."""
    import re
    txt = open(header_path).read()
    return sorted(set(re.findall(r"\b(letkf_[a-z_0-9]+)\s*\(", txt)))
