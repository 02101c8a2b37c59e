"""Seeded synthetic workloads for the visibility hot path.

This module is the one piece shared by the GPU path and its CPU checker.  It
holds configuration records and random draws only: antenna lattice
coordinates, channel centres, sidereal times, sky coefficients, gains and
unit-variance noise.  It performs none of the forward-model arithmetic
(no directions, beams, harmonics, fringes or likelihoods).

Every draw comes from ``numpy.random.Generator(PCG64(seed))`` in the fixed
order sky coefficients -> gains -> noise, so any consumer that asks for the
same config and seed sees bit-identical inputs.

Shapes follow the paper's mock observation (Sec. 3.1: a hexagonally packed
array with 14.6 m spacing, a 120-130 MHz band, a zenith-pointed drift scan
at latitude -30.7 deg) scaled to the workload sizes used here.  None of the
paper's data products (sky maps, 21 cm simulations, beams, mock visibilities)
are used: every input is synthetic.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

#: lattice spacing of the hex arrays (Sec. 3.1)
HEX_SPACING_M = 14.6
#: sidereal rotation rate, rad per solar second
OMEGA_EARTH = 7.2921159e-5


@dataclasses.dataclass(frozen=True)
class FieldConfig:
    """One observation: array, band, time span, sky grid and basis size."""

    name: str
    array: str                 # "hex" (side n) or "rhombus" (n x n)
    array_size: int
    n_freq: int
    freq_lo_hz: float
    freq_hi_hz: float
    n_time: int
    grid_nz: int               # rings, uniform in z = sin(dec)
    grid_nphi: int             # columns, uniform in right ascension
    lmax: int
    seed: int
    dt_s: float = 60.0
    lst0_rad: float = 0.0
    latitude_deg: float = -30.7
    spacing_m: float = HEX_SPACING_M
    fwhm_ref_deg: float = 10.0  # FWHM of the power beam at beam_ref_hz
    beam_ref_hz: float = 150e6
    gain_scatter: float = 0.05
    noise_frac: float = 0.01    # noise rms as a fraction of the visibility rms

    # -- derived sizes (pure bookkeeping) ---------------------------------
    @property
    def n_ant(self) -> int:
        return len(antenna_lattice(self))

    @property
    def n_bl(self) -> int:
        n = self.n_ant
        return n * (n - 1) // 2

    @property
    def n_pix(self) -> int:
        return self.grid_nz * self.grid_nphi

    @property
    def n_modes(self) -> int:
        return (self.lmax + 1) ** 2


def hex_lattice(side: int) -> np.ndarray:
    """Integer coordinates (i, j) of a centred hexagon of ``side`` antennas.

    Points of the triangular lattice with |i|, |j|, |i+j| <= side-1, ordered
    by j then i.  Sides 3/4/5/6/7 give 19/37/61/91/127 antennas.
    """
    r = side - 1
    pts = [(i, j) for j in range(-r, r + 1) for i in range(-r, r + 1)
           if abs(i + j) <= r]
    return np.asarray(pts, dtype=np.int64)


def rhombus_lattice(side: int) -> np.ndarray:
    """side x side rhombus on the triangular lattice, antenna index side*j+i."""
    pts = [(i, j) for j in range(side) for i in range(side)]
    return np.asarray(pts, dtype=np.int64)


def antenna_lattice(cfg: FieldConfig) -> np.ndarray:
    if cfg.array == "hex":
        return hex_lattice(cfg.array_size)
    if cfg.array == "rhombus":
        return rhombus_lattice(cfg.array_size)
    raise ValueError(f"unknown array kind {cfg.array!r}")


def lattice_basis(cfg: FieldConfig) -> np.ndarray:
    """Lattice basis vectors in ENU metres, shape [2][3]: e1 east, e2 at 60 deg."""
    a = cfg.spacing_m
    return np.array([[a, 0.0, 0.0],
                     [0.5 * a, 0.5 * math.sqrt(3.0) * a, 0.0]])


def antenna_enu(cfg: FieldConfig) -> np.ndarray:
    """Antenna positions [n_ant][3] in metres (coplanar, U = 0)."""
    ij = antenna_lattice(cfg).astype(np.float64)
    e = lattice_basis(cfg)
    return ij[:, :1] * e[0] + ij[:, 1:] * e[1]


def frequencies(cfg: FieldConfig) -> np.ndarray:
    """Channel centres in Hz: lo + (k + 1/2) * (hi - lo) / n."""
    k = np.arange(cfg.n_freq, dtype=np.float64)
    return cfg.freq_lo_hz + (k + 0.5) * (cfg.freq_hi_hz - cfg.freq_lo_hz) / cfg.n_freq


def lsts(cfg: FieldConfig) -> np.ndarray:
    """Local sidereal times in radians, one sample every dt_s solar seconds."""
    t = np.arange(cfg.n_time, dtype=np.float64)
    return cfg.lst0_rad + t * cfg.dt_s * OMEGA_EARTH


def latitude_rad(cfg: FieldConfig) -> float:
    return math.radians(cfg.latitude_deg)


def fwhm_ref_rad(cfg: FieldConfig) -> float:
    return math.radians(cfg.fwhm_ref_deg)


def mode_l(lmax: int) -> np.ndarray:
    """Degree l of every mode column, column index l*l + l + m."""
    return np.concatenate([np.full(2 * l + 1, l) for l in range(lmax + 1)])


@dataclasses.dataclass
class Draws:
    alm: np.ndarray        # [n_freq][n_modes] float64, a(lm, nu)
    alm_var: np.ndarray    # [n_freq][n_modes] float64, variance of the draw
    gains: np.ndarray      # [n_freq][n_ant] complex128
    noise_unit: np.ndarray  # [n_time][n_freq][n_bl] complex128, E|n|^2 = 1


def draw(cfg: FieldConfig, with_noise: bool = True) -> Draws:
    """All random inputs of one field, in the order sky -> gains -> noise.

    Sky: a0(lm) ~ N(0, (l+1)^-2.5), a(lm, nu) = a0(lm) (nu / 150 MHz)^-2.5.
    Gains: 1 + gain_scatter * CN(0,1), CN(0,1) = N(0,1/2) + i N(0,1/2).
    Noise: CN(0,1) per (time, channel, baseline); the caller scales it.
    """
    rng = np.random.Generator(np.random.PCG64(cfg.seed))
    ell = mode_l(cfg.lmax).astype(np.float64)
    var0 = (ell + 1.0) ** -2.5
    a0 = rng.standard_normal(cfg.n_modes) * np.sqrt(var0)
    scale = (frequencies(cfg) / 150e6) ** -2.5
    alm = scale[:, None] * a0[None, :]
    alm_var = (scale ** 2)[:, None] * var0[None, :]
    n_ant = cfg.n_ant
    g = rng.standard_normal((cfg.n_freq, n_ant, 2)) * math.sqrt(0.5)
    gains = 1.0 + cfg.gain_scatter * (g[..., 0] + 1j * g[..., 1])
    if with_noise:
        n = rng.standard_normal((cfg.n_time, cfg.n_freq, cfg.n_bl, 2)) * math.sqrt(0.5)
        noise = n[..., 0] + 1j * n[..., 1]
    else:
        noise = np.zeros((0,), dtype=np.complex128)
    return Draws(alm=alm, alm_var=alm_var, gains=gains, noise_unit=noise)


# -- the workloads --------------------------------------------------------
#: small case: 16-dish rhombus, 3072-pixel grid, lmax 20, 8 ch, 4 times
C0 = FieldConfig(name="c0_rhombus16_3072px_l20_8ch_4t", array="rhombus", array_size=4,
                 n_freq=8, freq_lo_hz=120e6, freq_hi_hz=180e6, n_time=4,
                 grid_nz=32, grid_nphi=96, lmax=20, seed=1000)
#: full case: 61-dish hex, 49152-pixel grid, lmax 100, 64 ch, 60 times
C1 = FieldConfig(name="c1_hex61_49152px_l100_64ch_60t", array="hex", array_size=5,
                 n_freq=64, freq_lo_hz=120e6, freq_hi_hz=130e6, n_time=60,
                 grid_nz=128, grid_nphi=384, lmax=100, seed=1001)


def serving_chain_config(c: int) -> FieldConfig:
    """Field of serving chain c: hex side from {3,4,5,7}, uneven band/time/lmax.

    Drawn from PCG64(2000 + c): hex side uniform on {3,4,5,7} (19/37/61/127
    antennas), n_freq uniform on [16,128], n_time uniform on [10,120],
    lmax uniform on [30,100]; shared 128 x 384 grid, 120-130 MHz band.
    """
    rng = np.random.Generator(np.random.PCG64(2000 + c))
    side = int(rng.choice([3, 4, 5, 7]))
    n_freq = int(rng.integers(16, 129))
    n_time = int(rng.integers(10, 121))
    lmax = int(rng.integers(30, 101))
    return FieldConfig(name=f"chain{c}", array="hex", array_size=side,
                       n_freq=n_freq, freq_lo_hz=120e6, freq_hi_hz=130e6,
                       n_time=n_time, grid_nz=128, grid_nphi=384, lmax=lmax,
                       seed=2000 + c)


def scaled(cfg: FieldConfig, **kw) -> FieldConfig:
    """A copy of ``cfg`` with some fields replaced (for small test cases)."""
    return dataclasses.replace(cfg, **kw)


__all__: List[str] = [
    "FieldConfig", "C0", "C1", "serving_chain_config", "scaled", "draw", "Draws",
    "antenna_lattice", "antenna_enu", "lattice_basis", "frequencies", "lsts",
    "latitude_rad", "fwhm_ref_rad", "mode_l", "hex_lattice", "rhombus_lattice",
    "HEX_SPACING_M", "OMEGA_EARTH",
]
