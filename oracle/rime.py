"""Directions, primary beam and the discrete RIME (oracle).

Sec. 2.1, eq. rime_discrete:
    V_b(nu, t) = dOmega sum_p K_pb A_p B_p,   K = exp(-2 pi i nu b . s_p(t) / c)
with A the shared power beam and B the sky.  The paper fixes the pixels on
the celestial sphere, so the fringe and the beam change with time
(eq. rime_matrix: one design matrix per time).  In this module's notation
S[t][nu][p] = dOmega * beam * sky is the per-pixel weight and the sum is
taken directly, in float64.

Topocentric direction of a celestial pixel (declination delta, right
ascension alpha) at local sidereal time LST and latitude phi, hour angle
H = LST - alpha (the textbook equatorial-to-horizon rotation):
    E = -cos(delta) sin(H)
    N =  cos(phi) sin(delta) - sin(phi) cos(delta) cos(H)
    U =  sin(phi) sin(delta) + cos(phi) cos(delta) cos(H)

Beam: a zenith-pointed Gaussian power beam, 1 at zenith (Sec. 3.4 fixes the
unit normalisation at boresight), zero at and below the horizon (the beam
covers the hemisphere above the horizon):
    B = exp(-theta^2 / (2 sigma^2)),  theta = arccos(U),
    sigma(nu) = F (nu_ref / nu) / (2 sqrt(2 ln 2)),
F = FWHM of the power beam at nu_ref, in radians.
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 299792458.0
FWHM_TO_SIGMA = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))


def enu_directions(dec: np.ndarray, ra: np.ndarray, lst: np.ndarray,
                   lat: float) -> np.ndarray:
    """Unit vectors [n_time][n_dir][3] (E, N, U) of fixed celestial directions."""
    dec = np.asarray(dec, dtype=np.float64)[None, :]
    ra = np.asarray(ra, dtype=np.float64)[None, :]
    h = np.asarray(lst, dtype=np.float64)[:, None] - ra
    cd, sd = np.cos(dec), np.sin(dec)
    cp, sp = math.cos(lat), math.sin(lat)
    e = -cd * np.sin(h)
    n = cp * sd - sp * cd * np.cos(h)
    u = sp * sd + cp * cd * np.cos(h)
    return np.stack([e, n, u], axis=-1)


def beam_sigma(freqs: np.ndarray, fwhm_ref: float, ref_hz: float) -> np.ndarray:
    return fwhm_ref * (ref_hz / np.asarray(freqs, dtype=np.float64)) * FWHM_TO_SIGMA


def beam(enu: np.ndarray, freqs: np.ndarray, fwhm_ref: float, ref_hz: float) -> np.ndarray:
    """B[t][nu][p] of the Gaussian power beam (zero where U <= 0)."""
    u = enu[..., 2]
    theta = np.arccos(np.clip(u, -1.0, 1.0))
    sig = beam_sigma(freqs, fwhm_ref, ref_hz)
    b = np.exp(-theta[:, None, :] ** 2 / (2.0 * sig[None, :, None] ** 2))
    return np.where(u[:, None, :] > 0.0, b, 0.0)


def dbeam_dfwhm(enu: np.ndarray, freqs: np.ndarray, fwhm_ref: float,
                ref_hz: float) -> np.ndarray:
    """dB/dF = B theta^2 / (sigma^2 F)  (sigma is proportional to F)."""
    u = enu[..., 2]
    theta = np.arccos(np.clip(u, -1.0, 1.0))
    sig = beam_sigma(freqs, fwhm_ref, ref_hz)
    b = beam(enu, freqs, fwhm_ref, ref_hz)
    return b * theta[:, None, :] ** 2 / (sig[None, :, None] ** 2 * fwhm_ref)


def vis_direct(bvec: np.ndarray, enu: np.ndarray, weight: np.ndarray,
               freqs: np.ndarray) -> np.ndarray:
    """V[t][nu][b] = sum_p weight[t][nu][p] exp(-2 pi i nu b . s_p(t) / c).

    Loop over (t, nu); the sum over directions is a matrix-vector product.
    Directions whose weight is zero at every channel of a time are dropped
    (their terms are exactly zero).
    """
    nt, nf = weight.shape[0], weight.shape[1]
    out = np.empty((nt, nf, bvec.shape[0]), dtype=np.complex128)
    for t in range(nt):
        keep = np.any(weight[t] != 0.0, axis=0)
        tau = bvec @ enu[t, keep].T / C_LIGHT          # [n_b][n_keep] seconds
        for f in range(nf):
            k = np.exp(-2j * math.pi * freqs[f] * tau)
            out[t, f] = k @ weight[t, f, keep]
    return out


def design_matrix(bvec: np.ndarray, enu_t: np.ndarray, beam_tf: np.ndarray,
                  nu: float, d_omega: float) -> np.ndarray:
    """Explicit A [n_b][n_pix] of eq. rime_matrix for one (t, nu): y = A x."""
    tau = bvec @ enu_t.T / C_LIGHT
    return d_omega * np.exp(-2j * math.pi * nu * tau) * beam_tf[None, :]


def fringe_adjoint(bvec: np.ndarray, enu: np.ndarray, omega: np.ndarray,
                   freqs: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Z[t][nu][p] = sum_b Re[omega[t][nu][b] exp(-2 pi i nu b . s_p(t) / c)].

    The transpose (over the reals) of ``vis_direct`` with respect to the
    weights: for real w, Re<omega*, V(w)> = <w, Z>.  Evaluated only where
    ``mask[t][p]`` is true (zero elsewhere).
    """
    nt, nf = omega.shape[0], omega.shape[1]
    out = np.zeros((nt, nf, enu.shape[1]))
    for t in range(nt):
        keep = mask[t]
        tau = bvec @ enu[t, keep].T / C_LIGHT
        for f in range(nf):
            k = np.exp(-2j * math.pi * freqs[f] * tau)
            out[t, f, keep] = np.real(omega[t, f] @ k)
    return out
