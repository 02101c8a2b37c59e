"""Python binding of libbayesvis (ctypes): argument marshalling only.

Every step of the visibility / chi^2 / gradient path runs in the HIP library;
this module checks shapes, dtypes and devices on the host, hands raw device
pointers and the current HIP stream to the C ABI, and raises on any non-zero
status.  PyTorch provides device memory and streams.  If the library is not
built, importing this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional

import numpy as np
import torch

from . import workload

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbayesvis.so")

VIS_FP32, VIS_BF16X3, VIS_FP16X3 = 1, 2, 3
VIS_SYNTH_DENSE, VIS_SYNTH_SEPARABLE = 0, 1
STORAGE_FOR = {VIS_FP32: 1, VIS_BF16X3: 2, VIS_FP16X3: 4}
STORAGE_SEPARABLE = 8   # factor tables of separable synthesis only


class VisError(RuntimeError):
    pass


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2504_07090_amd.build`")
    return C.CDLL(LIB_PATH)


_lib = _load()


class BasisDesc(C.Structure):
    _fields_ = [("grid_nz", C.c_int32), ("grid_nphi", C.c_int32), ("lmax", C.c_int32),
                ("storage", C.c_uint32)]


class FieldDesc(C.Structure):
    _fields_ = [("n_ant", C.c_int32), ("ant_lattice", C.POINTER(C.c_int32)),
                ("lattice_e1_m", C.c_double * 3), ("lattice_e2_m", C.c_double * 3),
                ("n_freq", C.c_int32), ("freq_hz", C.POINTER(C.c_double)),
                ("n_time", C.c_int32), ("lst_rad", C.POINTER(C.c_double)),
                ("latitude_rad", C.c_double), ("lmax", C.c_int32), ("beam_ref_hz", C.c_double),
                ("precision", C.c_int32), ("synthesis", C.c_int32)]


class FieldInfo(C.Structure):
    _fields_ = [("n_ant", C.c_int32), ("n_bl", C.c_int32), ("n_ubl", C.c_int32),
                ("n_freq", C.c_int32), ("n_time", C.c_int32), ("n_pix", C.c_int32),
                ("n_modes", C.c_int32), ("n_pix_visible", C.c_int32),
                ("lattice_extent", C.c_int32), ("precision", C.c_int32),
                ("synthesis", C.c_int32), ("d_omega", C.c_double), ("fwd_macs", C.c_double)]


_vp = C.c_void_p
_lib.vis_last_error.restype = C.c_char_p
_lib.vis_version.restype = C.c_char_p
_lib.vis_basis_workspace_bytes.argtypes = [C.POINTER(BasisDesc), C.POINTER(C.c_size_t)]
_lib.vis_basis_create.argtypes = [C.POINTER(BasisDesc), _vp, C.c_size_t, _vp, C.POINTER(_vp)]
_lib.vis_basis_destroy.argtypes = [_vp]
_lib.vis_field_workspace_bytes.argtypes = [_vp, C.POINTER(FieldDesc), C.POINTER(C.c_size_t)]
_lib.vis_field_create.argtypes = [_vp, C.POINTER(FieldDesc), _vp, C.c_size_t, _vp, C.POINTER(_vp)]
_lib.vis_field_get_info.argtypes = [_vp, C.POINTER(FieldInfo)]
_lib.vis_field_destroy.argtypes = [_vp]
_lib.vis_forward.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
_lib.vis_adjoint.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.chi2_and_grad.argtypes = [_vp, _vp, C.c_float, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
for _n in ("vis_basis_workspace_bytes", "vis_basis_create", "vis_basis_destroy",
           "vis_field_workspace_bytes", "vis_field_create", "vis_field_get_info",
           "vis_field_destroy", "vis_forward", "vis_adjoint", "chi2_and_grad"):
    getattr(_lib, _n).restype = C.c_int


def lib():
    return _lib


def _check(status: int, what: str):
    if status != 0:
        msg = _lib.vis_last_error().decode(errors="replace")
        raise VisError(f"{what} failed with status {status}: {msg}")


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, name: str, dtype, shape, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Basis:
    """Harmonic basis Y on the equal-area grid, generated on the GPU."""

    def __init__(self, grid_nz: int, grid_nphi: int, lmax: int, storage: int = 1,
                 device: str = "cuda"):
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.desc = BasisDesc(grid_nz, grid_nphi, lmax, storage)
        nbytes = C.c_size_t()
        _check(_lib.vis_basis_workspace_bytes(C.byref(self.desc), C.byref(nbytes)), "basis size")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        _check(_lib.vis_basis_create(C.byref(self.desc), _ptr(self.workspace), nbytes.value,
                                     C.c_void_p(_stream()), C.byref(h)), "vis_basis_create")
        self.handle = h
        self._lib = _lib
        self.grid_nz, self.grid_nphi, self.lmax, self.storage = grid_nz, grid_nphi, lmax, storage

    def __del__(self):
        # the library is held by the instance: module globals may already be
        # cleared when this runs at interpreter exit
        h, lib = getattr(self, "handle", None), getattr(self, "_lib", None)
        if h and lib is not None:
            lib.vis_basis_destroy(h)
            self.handle = None


class Field:
    """One observation (array, band, times) bound to a basis."""

    def __init__(self, basis: Basis, ant_lattice, e1, e2, freqs, lsts, latitude_rad: float,
                 lmax: int, beam_ref_hz: float = 150e6, precision: int = VIS_FP32,
                 synthesis: int = VIS_SYNTH_DENSE):
        self.basis = basis
        self.device = basis.device
        ant = np.ascontiguousarray(np.asarray(ant_lattice, dtype=np.int32).reshape(-1, 2))
        fr = np.ascontiguousarray(np.asarray(freqs, dtype=np.float64))
        ls = np.ascontiguousarray(np.asarray(lsts, dtype=np.float64))
        self._keep = (ant, fr, ls)
        d = FieldDesc()
        d.n_ant = len(ant)
        d.ant_lattice = ant.ctypes.data_as(C.POINTER(C.c_int32))
        d.lattice_e1_m = (C.c_double * 3)(*[float(x) for x in e1])
        d.lattice_e2_m = (C.c_double * 3)(*[float(x) for x in e2])
        d.n_freq = len(fr)
        d.freq_hz = fr.ctypes.data_as(C.POINTER(C.c_double))
        d.n_time = len(ls)
        d.lst_rad = ls.ctypes.data_as(C.POINTER(C.c_double))
        d.latitude_rad = float(latitude_rad)
        d.lmax = int(lmax)
        d.beam_ref_hz = float(beam_ref_hz)
        d.precision = int(precision)
        d.synthesis = int(synthesis)
        self.desc = d
        nbytes = C.c_size_t()
        _check(_lib.vis_field_workspace_bytes(basis.handle, C.byref(d), C.byref(nbytes)),
               "field size")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        _check(_lib.vis_field_create(basis.handle, C.byref(d), _ptr(self.workspace), nbytes.value,
                                     C.c_void_p(_stream()), C.byref(h)), "vis_field_create")
        self.handle = h
        self._lib = _lib
        info = FieldInfo()
        _check(_lib.vis_field_get_info(h, C.byref(info)), "vis_field_get_info")
        self.info = info
        self.n_ant, self.n_bl, self.n_ubl = info.n_ant, info.n_bl, info.n_ubl
        self.n_freq, self.n_time, self.n_modes = info.n_freq, info.n_time, info.n_modes
        self.precision = precision
        self.synthesis = synthesis

    @classmethod
    def from_config(cls, basis: Basis, cfg: workload.FieldConfig, precision: int = VIS_FP32,
                    synthesis: int = VIS_SYNTH_DENSE):
        e = workload.lattice_basis(cfg)
        return cls(basis, workload.antenna_lattice(cfg), e[0], e[1], workload.frequencies(cfg),
                   workload.lsts(cfg), workload.latitude_rad(cfg), cfg.lmax, cfg.beam_ref_hz,
                   precision, synthesis)

    @property
    def fwd_macs(self) -> float:
        """Complex x real MACs of one fringe pass (unique baselines, pixels above the horizon)."""
        return float(self.info.fwd_macs)

    def __del__(self):
        h, lib = getattr(self, "handle", None), getattr(self, "_lib", None)
        if h and lib is not None:
            lib.vis_field_destroy(h)
            self.handle = None

    # -- argument checks -----------------------------------------------------
    def _params(self, alm, gains, fwhm):
        dev = self.device
        _need(alm, "alm", torch.float32, (self.n_freq, self.n_modes), dev)
        _need(gains, "gains", torch.complex64, (self.n_freq, self.n_ant), dev)
        _need(fwhm, "fwhm", torch.float32, (1,), dev)

    def _vis_shape(self):
        return (self.n_time, self.n_freq, self.n_bl)


def basis_for(cfg: workload.FieldConfig, storage: int = 1, device: str = "cuda") -> Basis:
    return Basis(cfg.grid_nz, cfg.grid_nphi, cfg.lmax, storage, device)


def forward(field: Field, alm, gains, fwhm) -> torch.Tensor:
    """Model visibilities m[t][nu][bl] (complex64)."""
    field._params(alm, gains, fwhm)
    vis = torch.empty(field._vis_shape(), dtype=torch.complex64, device=field.device)
    _check(_lib.vis_forward(field.handle, _ptr(alm), _ptr(gains), _ptr(fwhm), _ptr(vis),
                            C.c_void_p(_stream())), "vis_forward")
    return vis


def adjoint(field: Field, alm, gains, fwhm, dvis):
    """(dL/da, dL/dg, dL/dF) given dvis = dL/dRe m + i dL/dIm m."""
    field._params(alm, gains, fwhm)
    _need(dvis, "dvis", torch.complex64, field._vis_shape(), field.device)
    ga = torch.empty_like(alm)
    gg = torch.empty_like(gains)
    gf = torch.empty_like(fwhm)
    _check(_lib.vis_adjoint(field.handle, _ptr(alm), _ptr(gains), _ptr(fwhm), _ptr(dvis),
                            _ptr(ga), _ptr(gg), _ptr(gf), C.c_void_p(_stream())), "vis_adjoint")
    return ga, gg, gf


def chi2_and_grad(field: Field, data, sigma_n: float, alm, gains, fwhm, grads: bool = True):
    """(chi2 as a 0-d float64 tensor, dchi2/da, dchi2/dg, dchi2/dF)."""
    field._params(alm, gains, fwhm)
    _need(data, "data", torch.complex64, field._vis_shape(), field.device)
    if not (sigma_n > 0 and math.isfinite(sigma_n)):
        raise ValueError("sigma_n must be positive and finite")
    x2 = torch.empty((), dtype=torch.float64, device=field.device)
    if grads:
        ga, gg, gf = torch.empty_like(alm), torch.empty_like(gains), torch.empty_like(fwhm)
    else:
        ga = gg = gf = None
    _check(_lib.chi2_and_grad(field.handle, _ptr(data), C.c_float(sigma_n), _ptr(alm), _ptr(gains),
                              _ptr(fwhm), _ptr(x2), _ptr(ga), _ptr(gg), _ptr(gf),
                              C.c_void_p(_stream())), "chi2_and_grad")
    return x2, ga, gg, gf


class VisChi2Function(torch.autograd.Function):
    """chi^2(a, g, F) with the hand-written adjoint as its backward.

    forward runs chi2_and_grad (forward model, chi^2 and the adjoint in one
    sequence) and keeps only the gradients; backward scales them by the
    incoming scalar cotangent.  Gains are complex64; their gradient follows
    PyTorch's convention for real losses (conjugate Wirtinger, i.e.
    dL/dRe g + i dL/dIm g).
    """

    @staticmethod
    def forward(ctx, alm, gains, fwhm, field: Field, data, sigma_n: float):
        x2, ga, gg, gf = chi2_and_grad(field, data, sigma_n, alm.detach(), gains.detach(),
                                       fwhm.detach(), grads=True)
        ctx.save_for_backward(ga, gg, gf)
        return x2

    @staticmethod
    def backward(ctx, gout):
        ga, gg, gf = ctx.saved_tensors
        s = gout.to(torch.float32)
        return ga * s, gg * s, gf * s, None, None, None


# -------------------------------------------------------------------- map-making --
_lib.vis_make_map.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]


def make_map(field: Field, data, gains, fwhm, with_weight: bool = True):
    """(map [n_freq][n_pix], weight [n_freq][n_pix] or None): Re(A^H y) / diag(A^H A)."""
    dev = field.device
    _need(gains, "gains", torch.complex64, (field.n_freq, field.n_ant), dev)
    _need(fwhm, "fwhm", torch.float32, (1,), dev)
    _need(data, "data", torch.complex64, field._vis_shape(), dev)
    npix = field.info.n_pix
    out = torch.empty((field.n_freq, npix), dtype=torch.float32, device=dev)
    wgt = torch.empty_like(out) if with_weight else None
    _check(_lib.vis_make_map(field.handle, _ptr(data), _ptr(gains), _ptr(fwhm), _ptr(out), _ptr(wgt),
                             C.c_void_p(_stream())), "vis_make_map")
    return out, wgt


# ------------------------------------------------------------------ delay filter --
_dp = C.POINTER(C.c_double)
_lib.vis_filter_build.argtypes = [C.c_int32, _dp, C.c_double, C.c_double, _dp, _dp]
_lib.vis_filter_workspace_bytes.argtypes = [C.c_int32, C.POINTER(C.c_size_t)]
_lib.vis_filter_create.argtypes = [C.c_int32, _dp, C.c_double, C.c_double, _vp, C.c_size_t, _vp,
                                   C.POINTER(_vp)]
_lib.vis_filter_destroy.argtypes = [_vp]
_lib.vis_filtered_work_bytes.argtypes = [_vp, C.POINTER(C.c_size_t)]
_lib.chi2_filtered_and_grad.argtypes = [_vp, _vp, _vp, C.c_float, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                        _vp, C.c_size_t, _vp]
_lib.chi2_filtered_and_grad_noalloc.argtypes = [_vp, _vp, _vp, C.c_float, _vp, _vp, _vp, _vp, _vp,
                                                _vp, _vp, _vp]


def filter_build(freqs, tau_max: float = 250e-9, noise_ratio: float = 1e-8):
    """The library's delay filter F and diag(F F^T), computed on the host (FP64)."""
    fr = np.ascontiguousarray(np.asarray(freqs, dtype=np.float64))
    n = len(fr)
    f = np.empty((n, n), dtype=np.float64)
    d = np.empty(n, dtype=np.float64)
    _check(_lib.vis_filter_build(n, fr.ctypes.data_as(_dp), float(tau_max), float(noise_ratio),
                                 f.ctypes.data_as(_dp), d.ctypes.data_as(_dp)), "vis_filter_build")
    return f, d


class Filter:
    """Delay filter of one channel list, resident on the device."""

    def __init__(self, freqs, tau_max: float = 250e-9, noise_ratio: float = 1e-8,
                 device: str = "cuda"):
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        fr = np.ascontiguousarray(np.asarray(freqs, dtype=np.float64))
        nbytes = C.c_size_t()
        _check(_lib.vis_filter_workspace_bytes(len(fr), C.byref(nbytes)), "filter size")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        _check(_lib.vis_filter_create(len(fr), fr.ctypes.data_as(_dp), float(tau_max),
                                      float(noise_ratio), _ptr(self.workspace), nbytes.value,
                                      C.c_void_p(_stream()), C.byref(h)), "vis_filter_create")
        self.handle = h
        self._lib = _lib
        self.n_freq = len(fr)

    def __del__(self):
        h, lib = getattr(self, "handle", None), getattr(self, "_lib", None)
        if h and lib is not None:
            lib.vis_filter_destroy(h)
            self.handle = None


def chi2_filtered_and_grad(field: Field, filt: Filter, data, sigma_n: float, alm, gains, fwhm,
                           grads: bool = True):
    """(chi^2_F as a 0-d float64 tensor, gradients) of the delay-filtered likelihood."""
    field._params(alm, gains, fwhm)
    _need(data, "data", torch.complex64, field._vis_shape(), field.device)
    if not (sigma_n > 0 and math.isfinite(sigma_n)):
        raise ValueError("sigma_n must be positive and finite")
    nbytes = C.c_size_t()
    _check(_lib.vis_filtered_work_bytes(field.handle, C.byref(nbytes)), "filtered work size")
    work = torch.empty(nbytes.value, dtype=torch.uint8, device=field.device)
    x2 = torch.empty((), dtype=torch.float64, device=field.device)
    if grads:
        ga, gg, gf = torch.empty_like(alm), torch.empty_like(gains), torch.empty_like(fwhm)
    else:
        ga = gg = gf = None
    _check(_lib.chi2_filtered_and_grad(field.handle, filt.handle, _ptr(data), C.c_float(sigma_n),
                                       _ptr(alm), _ptr(gains), _ptr(fwhm), _ptr(x2), _ptr(ga),
                                       _ptr(gg), _ptr(gf), _ptr(work), nbytes.value,
                                       C.c_void_p(_stream())), "chi2_filtered_and_grad")
    return x2, ga, gg, gf


def chi2_filtered_and_grad_noalloc(field: Field, filt: Filter, data, sigma_n: float, alm, gains,
                                   fwhm, out=None, grads: bool = True):
    """chi2_filtered_and_grad through the entry point that allocates nothing: its
    scratch is the library's static per-GPU array.  ``out`` = (chi2, ga, gg, gf)
    preallocated outputs (any gradient may be None); allocated here if omitted."""
    field._params(alm, gains, fwhm)
    _need(data, "data", torch.complex64, field._vis_shape(), field.device)
    if not (sigma_n > 0 and math.isfinite(sigma_n)):
        raise ValueError("sigma_n must be positive and finite")
    if out is None:
        x2 = torch.empty((), dtype=torch.float64, device=field.device)
        if grads:
            ga, gg, gf = torch.empty_like(alm), torch.empty_like(gains), torch.empty_like(fwhm)
        else:
            ga = gg = gf = None
    else:
        x2, ga, gg, gf = out
    _check(_lib.chi2_filtered_and_grad_noalloc(field.handle, filt.handle, _ptr(data),
                                               C.c_float(sigma_n), _ptr(alm), _ptr(gains),
                                               _ptr(fwhm), _ptr(x2), _ptr(ga), _ptr(gg), _ptr(gf),
                                               C.c_void_p(_stream())),
           "chi2_filtered_and_grad_noalloc")
    return x2, ga, gg, gf


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("total_ms", C.c_double)]


_lib.vis_profile_enable.argtypes = [_vp, C.c_int32]
_lib.vis_profile_enable.restype = C.c_int
_lib.vis_profile_read.argtypes = [_vp, C.POINTER(KernelTime), C.c_int32, C.POINTER(C.c_int32),
                                  C.c_int32]
_lib.vis_profile_read.restype = C.c_int


def profile_enable(field: Field, on: bool = True):
    _check(_lib.vis_profile_enable(field.handle, 1 if on else 0), "vis_profile_enable")


def profile_read(field: Field, reset: bool = False):
    """{kernel name: (launches, total ms)} accumulated while profiling was on."""
    buf = (KernelTime * 64)()
    n = C.c_int32()
    _check(_lib.vis_profile_read(field.handle, buf, 64, C.byref(n), 1 if reset else 0),
           "vis_profile_read")
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms))
            for i in range(n.value)}
