"""Delay (high-pass) filter along frequency and the filtered likelihood (oracle).

Sec. 2.1, eq. rime_filter: model and data are both multiplied along the
frequency axis by a real N_freq x N_freq matrix F before they are compared.
Eq. gpr: F = I - C_fg (C_fg + C_noise)^-1, where the foreground covariance
C_fg is a sinc in frequency difference (the transform of a tophat of
half-width tau_max in delay) and C_noise is diagonal, noise_ratio times the
amplitude of C_fg.  Sec. 3.5, eq. filtered_noise: the filtered noise has
covariance N~ = F N F^T; the likelihood keeps only its diagonal,
    chi^2_F = sum_{t, nu, bl} |(F (d - m))_nu|^2 / N~_nu,nu,
with N = sigma_n^2 I per real component, so N~_nu,nu = sigma_n^2 (F F^T)_nu,nu.
The cotangent of the model visibilities is c = -2 F^T ((F (d - m)) / N~),
and the parameter gradients follow from the same adjoint as the plain chi^2.

Readings: sinc(x) = sin(pi x) / (pi x); C_fg(nu, nu') = sinc(2 tau_max (nu - nu'))
(unit amplitude, so C_noise = noise_ratio I); tau_max = 250 ns and
noise_ratio = 1e-8 as in the paper.
"""
from __future__ import annotations

import numpy as np

from . import model


def sinc_covariance(freqs: np.ndarray, tau_max: float) -> np.ndarray:
    """C_fg[i][j] = sinc(2 tau_max (nu_i - nu_j)), the tophat-in-delay covariance."""
    d = np.subtract.outer(freqs, freqs)
    return np.sinc(2.0 * tau_max * d)


def delay_filter(freqs: np.ndarray, tau_max: float = 250e-9, noise_ratio: float = 1e-8) -> np.ndarray:
    """F = I - C_fg (C_fg + noise_ratio I)^-1 (eq. gpr), float64."""
    c = sinc_covariance(freqs, tau_max)
    n = len(freqs)
    k = c + noise_ratio * np.eye(n)
    # C (C + eps I)^-1 = ((C + eps I)^-1 C)^T for symmetric C
    return np.eye(n) - np.linalg.solve(k, c).T


def filtered_noise_diag(f: np.ndarray, sigma_n: float) -> np.ndarray:
    """Diagonal of N~ = F N F^T with N = sigma_n^2 I (eq. filtered_noise)."""
    return sigma_n ** 2 * np.sum(f * f, axis=1)


def chi2_filtered(field: model.Field, data, sigma_n, f, alm, gains, fwhm) -> float:
    m = model.forward(field, alm, gains, fwhm)
    rf = np.einsum("ij,tjb->tib", f, data - m)
    w = 1.0 / filtered_noise_diag(f, sigma_n)
    return float(np.sum(np.abs(rf) ** 2 * w[None, :, None]))


def chi2_filtered_and_grad(field: model.Field, data, sigma_n, f, alm, gains, fwhm):
    """(chi^2_F, dchi^2_F/da, dchi^2_F/dg, dchi^2_F/dF) over all channels."""
    m = model.forward(field, alm, gains, fwhm)
    rf = np.einsum("ij,tjb->tib", f, data - m)
    w = 1.0 / filtered_noise_diag(f, sigma_n)
    wr = rf * w[None, :, None]
    x2 = float(np.sum(np.abs(rf) ** 2 * w[None, :, None]))
    cot = -2.0 * np.einsum("ji,tjb->tib", f, wr)
    ga, gg, gfw = model.adjoint(field, alm, gains, fwhm, cot)
    return x2, ga, gg, gfw
