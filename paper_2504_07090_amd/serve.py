"""Python binding of the HMC server (ctypes): argument marshalling only.

The server keeps every chain's state in a caller-provided device arena and
runs leapfrog steps as batched kernel launches on a worker thread inside the
library.  Helpers here pack parameter vectors in the server's layout and call
the library's mass-matrix set-up (hmc_mass_diag, hmc_gain_mass_blocks).
"""
from __future__ import annotations

import ctypes as C
import math
from typing import List, Optional

import numpy as np
import torch

from . import vis as V

_lib = V.lib()
_vp = C.c_void_p


class ServerConfig(C.Structure):
    _fields_ = [("max_chains", C.c_int32), ("max_batch", C.c_int32), ("batched", C.c_int32),
                ("inflight_ticks", C.c_int32)]


class ChainInit(C.Structure):
    _fields_ = [("field", _vp), ("data", _vp), ("sigma_n", C.c_float), ("q0", _vp),
                ("minv", _vp), ("alm_prior_var", _vp), ("gain_prior_sigma", C.c_float),
                ("eps", C.c_float), ("n_leapfrog", C.c_int32), ("adapt_step", C.c_int32),
                ("seed", C.c_uint64), ("stream_id", C.c_uint32), ("gain_chol", _vp),
                ("nuts_max_depth", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("chain", C.c_int32), ("trajectory", C.c_int32), ("accepted", C.c_int32),
                ("status", C.c_int32), ("h0", C.c_double), ("h1", C.c_double),
                ("chi2", C.c_double), ("eps", C.c_float), ("n_grad", C.c_int32),
                ("t_submit_ns", C.c_uint64), ("t_done_ns", C.c_uint64), ("tree_depth", C.c_int32),
                ("accept_stat", C.c_float)]


class Stats(C.Structure):
    _fields_ = [("requests", C.c_int64), ("p10_ms", C.c_double), ("p50_ms", C.c_double),
                ("p90_ms", C.c_double), ("p99_ms", C.c_double), ("max_ms", C.c_double), ("arena_free_bytes", C.c_int64), ("live_chains", C.c_int32)]


for _n in ("hmc_chain_footprint_bytes", "hmc_chain_footprint_dense_gain_bytes",
           "hmc_chain_footprint_nuts_bytes", "hmc_chain_footprint_nuts_dense_gain_bytes"):
    getattr(_lib, _n).argtypes = [_vp]
    getattr(_lib, _n).restype = C.c_size_t
_lib.hmc_mass_work_bytes.argtypes = [_vp, C.POINTER(C.c_size_t)]
_lib.hmc_mass_diag.argtypes = [_vp, _vp, _vp, _vp, C.c_float, _vp, C.c_float, C.c_int32,
                               C.c_uint64, _vp, _vp, _vp, C.c_size_t, _vp]
_lib.hmc_gain_mass_blocks.argtypes = [_vp, _vp, _vp, _vp, C.c_float, C.c_float, _vp, _vp,
                                      C.c_size_t, _vp]
_lib.hmc_server_create.argtypes = [C.POINTER(ServerConfig), _vp, C.c_size_t, _vp, C.POINTER(_vp)]
_lib.hmc_chain_admit.argtypes = [_vp, C.POINTER(ChainInit), C.POINTER(C.c_int32)]
_lib.hmc_submit.argtypes = [_vp, C.c_int32, C.c_int32]
_lib.hmc_poll.argtypes = [_vp, C.POINTER(Result), C.c_int32, C.POINTER(C.c_int32), C.c_int32]
_lib.hmc_chain_position.argtypes = [_vp, C.c_int32, _vp, _vp]
_lib.hmc_chain_release.argtypes = [_vp, C.c_int32]
_lib.hmc_server_stats.argtypes = [_vp, C.POINTER(Stats), C.c_int32]
_lib.hmc_server_destroy.argtypes = [_vp]
for _n in ("hmc_mass_work_bytes", "hmc_mass_diag", "hmc_gain_mass_blocks", "hmc_server_create",
           "hmc_chain_admit", "hmc_submit", "hmc_poll", "hmc_chain_position",
           "hmc_chain_release", "hmc_server_stats", "hmc_server_destroy"):
    getattr(_lib, _n).restype = C.c_int

VIS_EAGAIN, VIS_ENUMERIC = -4, -6


class Layout:
    """Offsets of the parameter vector: [a | pad | gains (Re, Im) | F]."""

    def __init__(self, field: V.Field):
        self.nalm = field.n_freq * field.n_modes
        self.goff = (self.nalm + 63) // 64 * 64
        self.ngain = 2 * field.n_freq * field.n_ant
        self.length = self.goff + self.ngain + 1
        self.shape = (field.n_freq, field.n_modes, field.n_ant)

    def pack(self, alm: torch.Tensor, gains: torch.Tensor, fwhm: torch.Tensor) -> torch.Tensor:
        q = torch.zeros(self.length, dtype=torch.float32, device=alm.device)
        q[:self.nalm] = alm.reshape(-1)
        q[self.goff:self.goff + self.ngain] = torch.view_as_real(gains).reshape(-1)
        q[-1] = fwhm.reshape(-1)[0]
        return q

    def unpack(self, q: torch.Tensor):
        nf, nm, na = self.shape
        alm = q[:self.nalm].reshape(nf, nm)
        g = torch.view_as_complex(q[self.goff:self.goff + self.ngain].reshape(nf, na, 2).contiguous())
        return alm, g, q[-1:]


def _mass_work(field: V.Field) -> torch.Tensor:
    n = C.c_size_t()
    V._check(_lib.hmc_mass_work_bytes(field.handle, C.byref(n)), "hmc_mass_work_bytes")
    return torch.empty(n.value, dtype=torch.uint8, device=field.device)


def mass_diag(field: V.Field, alm, gains, fwhm, sigma_n: float,
              alm_prior_var: Optional[torch.Tensor] = None, gain_prior_sigma: float = 0.0,
              n_probes: int = 8, seed: int = 0):
    """(hdiag, minv) in the server's parameter layout from hmc_mass_diag: the
    Gauss-Newton diagonal of chi^2 / 2 (Hutchinson probes for the sky and F,
    exact for the gains) plus the prior precisions, and its inverse."""
    lay = Layout(field)
    V._need(alm, "alm", torch.float32, (field.n_freq, field.n_modes), field.device)
    V._need(gains, "gains", torch.complex64, (field.n_freq, field.n_ant), field.device)
    V._need(fwhm, "fwhm", torch.float32, (1,), field.device)
    if alm_prior_var is not None:
        V._need(alm_prior_var, "alm_prior_var", torch.float32, (field.n_freq, field.n_modes),
                field.device)
    work = _mass_work(field)
    h = torch.empty(lay.length, dtype=torch.float32, device=field.device)
    minv = torch.empty_like(h)
    V._check(_lib.hmc_mass_diag(field.handle, V._ptr(alm), V._ptr(gains), V._ptr(fwhm), sigma_n,
                                V._ptr(alm_prior_var), gain_prior_sigma, n_probes, seed, V._ptr(h),
                                V._ptr(minv), V._ptr(work), work.numel(), C.c_void_p(V._stream())),
             "hmc_mass_diag")
    return h, minv


def gain_mass_blocks(field: V.Field, alm, gains, fwhm, sigma_n: float,
                     gain_prior_sigma: float) -> torch.Tensor:
    """Cholesky factors [n_freq][2 n_ant][2 n_ant] (float32, device) of the dense
    per-channel gain mass blocks from hmc_gain_mass_blocks: the Gauss-Newton gain
    Hessian of chi^2 / 2 plus 2 / s_g^2 I (App. B)."""
    V._need(alm, "alm", torch.float32, (field.n_freq, field.n_modes), field.device)
    V._need(gains, "gains", torch.complex64, (field.n_freq, field.n_ant), field.device)
    V._need(fwhm, "fwhm", torch.float32, (1,), field.device)
    work = _mass_work(field)
    nb = 2 * field.n_ant
    chol = torch.empty(field.n_freq, nb, nb, dtype=torch.float32, device=field.device)
    V._check(_lib.hmc_gain_mass_blocks(field.handle, V._ptr(alm), V._ptr(gains), V._ptr(fwhm),
                                       sigma_n, gain_prior_sigma, V._ptr(chol), V._ptr(work),
                                       work.numel(), C.c_void_p(V._stream())),
             "hmc_gain_mass_blocks")
    return chol


class Server:
    def __init__(self, arena_bytes: int, max_chains: int = 64, max_batch: int = 64,
                 batched: int = 1, device: str = "cuda", inflight_ticks: int = 1):
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        self.stream = torch.cuda.Stream(device=self.arena.device)
        cfg = ServerConfig(max_chains, max_batch, batched, inflight_ticks)
        h = C.c_void_p()
        V._check(_lib.hmc_server_create(C.byref(cfg), C.c_void_p(self.arena.data_ptr()),
                                        self.arena.numel(), C.c_void_p(self.stream.cuda_stream),
                                        C.byref(h)), "hmc_server_create")
        self.handle = h
        self._keep = {}

    @staticmethod
    def footprint(field: V.Field, dense_gains: bool = False, nuts: bool = False) -> int:
        if nuts and dense_gains:
            return int(_lib.hmc_chain_footprint_nuts_dense_gain_bytes(field.handle))
        if nuts:
            return int(_lib.hmc_chain_footprint_nuts_bytes(field.handle))
        if dense_gains:
            return int(_lib.hmc_chain_footprint_dense_gain_bytes(field.handle))
        return int(_lib.hmc_chain_footprint_bytes(field.handle))

    def admit(self, field: V.Field, data: torch.Tensor, sigma_n: float, q0: torch.Tensor,
              minv: torch.Tensor, alm_prior_var: torch.Tensor, gain_prior_sigma: float,
              eps: float, n_leapfrog: int, seed: int, stream_id: int,
              adapt_step: bool = False, gain_chol: Optional[torch.Tensor] = None,
              nuts_max_depth: int = 0) -> Optional[int]:
        """Chain id, or None if the arena has no room now (VIS_EAGAIN).
        gain_chol: optional [n_freq][2 n_ant][2 n_ant] lower Cholesky factors of
        dense per-channel gain mass blocks.  nuts_max_depth > 0: No-U-Turn
        trajectories of at most that many doublings (n_leapfrog ignored)."""
        lay = Layout(field)
        V._need(data, "data", torch.complex64, (field.n_time, field.n_freq, field.n_bl), field.device)
        V._need(q0, "q0", torch.float32, (lay.length,), field.device)
        V._need(minv, "minv", torch.float32, (lay.length,), field.device)
        V._need(alm_prior_var, "alm_prior_var", torch.float32, (field.n_freq, field.n_modes),
                field.device)
        if gain_chol is not None:
            V._need(gain_chol, "gain_chol", torch.float32,
                    (field.n_freq, 2 * field.n_ant, 2 * field.n_ant), field.device)
        torch.cuda.current_stream().synchronize()
        init = ChainInit(field.handle, data.data_ptr(), sigma_n, q0.data_ptr(), minv.data_ptr(),
                         alm_prior_var.data_ptr(), gain_prior_sigma, eps, n_leapfrog,
                         1 if adapt_step else 0, seed, stream_id,
                         None if gain_chol is None else gain_chol.data_ptr(), nuts_max_depth)
        cid = C.c_int32()
        st = _lib.hmc_chain_admit(self.handle, C.byref(init), C.byref(cid))
        if st == VIS_EAGAIN:
            return None
        V._check(st, "hmc_chain_admit")
        self._keep[cid.value] = (field, data)
        return cid.value

    def submit(self, chain: int, n_traj: int):
        V._check(_lib.hmc_submit(self.handle, chain, n_traj), "hmc_submit")

    def poll(self, max_results: int = 256, timeout_ms: int = 0) -> List[dict]:
        buf = (Result * max_results)()
        n = C.c_int32()
        V._check(_lib.hmc_poll(self.handle, buf, max_results, C.byref(n), timeout_ms), "hmc_poll")
        return [{f: getattr(buf[i], f) for f, _ in Result._fields_} for i in range(n.value)]

    def position(self, chain: int, length: int, device) -> torch.Tensor:
        q = torch.empty(length, dtype=torch.float32, device=device)
        V._check(_lib.hmc_chain_position(self.handle, chain, C.c_void_p(q.data_ptr()), None),
                 "hmc_chain_position")
        return q

    def release(self, chain: int):
        V._check(_lib.hmc_chain_release(self.handle, chain), "hmc_chain_release")
        self._keep.pop(chain, None)

    def stats(self, reset: bool = False) -> dict:
        s = Stats()
        V._check(_lib.hmc_server_stats(self.handle, C.byref(s), 1 if reset else 0), "hmc_server_stats")
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def close(self):
        h = getattr(self, "handle", None)
        if h:
            V._check(_lib.hmc_server_destroy(h), "hmc_server_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def wait(self, n_results: int, timeout_s: float = 120.0) -> List[dict]:
        """Collect n_results trajectory results (raises on timeout)."""
        import time
        out: List[dict] = []
        t_end = time.monotonic() + timeout_s
        while len(out) < n_results:
            if time.monotonic() > t_end:
                raise TimeoutError(f"only {len(out)} of {n_results} results")
            out += self.poll(256, timeout_ms=100)
        return out
