"""Sky pixelisation and real spherical-harmonic synthesis (oracle).

Sec. 2.1 / Sec. 3.2: the sky is pixelised on an equal-area rectangular grid
in right ascension and declination; pixels carry flux per solid angle times
the pixel solid angle.  Here: N_z rings uniform in z = sin(dec) with centres
z_j = -1 + (j + 1/2) 2/N_z, N_phi columns alpha_k = (k + 1/2) 2 pi / N_phi,
pixel index p = j N_phi + k, solid angle dOmega = 4 pi / (N_z N_phi).

Sec. 3.2 (eq. fg_harmonics, eq. fg_harmonic_matrix) writes the sky as a
harmonic synthesis I = Y a.  Here Y holds real, orthonormal full-sky
harmonics with integer l (the orthonormality of App. A, eq. sht_ortho),
column l*l + l + m, no Condon-Shortley phase:
    m = 0:  lambda_l0(z)
    m > 0:  sqrt(2) lambda_lm(z) cos(m alpha)
    m < 0:  sqrt(2) lambda_l|m|(z) sin(|m| alpha)
with lambda_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) P_l^m.  The normalised
functions are built by the standard stable three-term recurrence in l,
which never forms the factorials (App. A discusses why unnormalised
high-order Legendre functions overflow).
"""
from __future__ import annotations

import math

import numpy as np


def grid(nz: int, nphi: int):
    """Ring centres z_j, column centres alpha_k and pixel solid angle."""
    z = -1.0 + (np.arange(nz) + 0.5) * 2.0 / nz
    alpha = (np.arange(nphi) + 0.5) * 2.0 * math.pi / nphi
    d_omega = 4.0 * math.pi / (nz * nphi)
    return z, alpha, d_omega


def pixel_dec_ra(nz: int, nphi: int):
    """Declination and right ascension of every pixel, index j*nphi + k."""
    z, alpha, _ = grid(nz, nphi)
    dec = np.arcsin(z)
    return np.repeat(dec, nphi), np.tile(alpha, nz)


def legendre_normalized(lmax: int, z: np.ndarray) -> np.ndarray:
    """lambda_lm(z) for 0 <= m <= l <= lmax, shape [len(z)][lmax+1][lmax+1] ([.., l, m]).

    lambda_00 = 1/sqrt(4 pi);
    lambda_mm = sqrt((2m+1)/(2m)) sqrt(1-z^2) lambda_{m-1,m-1};
    lambda_{m+1,m} = sqrt(2m+3) z lambda_mm;
    lambda_lm = sqrt((4l^2-1)/(l^2-m^2)) [z lambda_{l-1,m}
                 - sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)) lambda_{l-2,m}].
    """
    z = np.asarray(z, dtype=np.float64)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    lam = np.zeros((z.size, lmax + 1, lmax + 1))
    lam[:, 0, 0] = 1.0 / math.sqrt(4.0 * math.pi)
    for m in range(1, lmax + 1):
        lam[:, m, m] = math.sqrt((2 * m + 1) / (2.0 * m)) * s * lam[:, m - 1, m - 1]
    for m in range(0, lmax):
        lam[:, m + 1, m] = math.sqrt(2 * m + 3) * z * lam[:, m, m]
    for m in range(0, lmax + 1):
        for l in range(m + 2, lmax + 1):
            a = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            b = math.sqrt(((l - 1) ** 2 - m * m) / (4.0 * (l - 1) ** 2 - 1.0))
            lam[:, l, m] = a * (z * lam[:, l - 1, m] - b * lam[:, l - 2, m])
    return lam


def real_ylm(lmax: int, z: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Real orthonormal Y at points (z, phi), shape [npts][(lmax+1)^2]."""
    z = np.asarray(z, dtype=np.float64).ravel()
    phi = np.asarray(phi, dtype=np.float64).ravel()
    lam = legendre_normalized(lmax, z)
    out = np.empty((z.size, (lmax + 1) ** 2))
    r2 = math.sqrt(2.0)
    for l in range(lmax + 1):
        c = l * l + l
        out[:, c] = lam[:, l, 0]
        for m in range(1, l + 1):
            out[:, c + m] = r2 * lam[:, l, m] * np.cos(m * phi)
            out[:, c - m] = r2 * lam[:, l, m] * np.sin(m * phi)
    return out


def basis_matrix(nz: int, nphi: int, lmax: int) -> np.ndarray:
    """Y [n_pix][n_modes] on the grid (memory n_pix * n_modes * 8 bytes)."""
    dec, ra = pixel_dec_ra(nz, nphi)
    return real_ylm(lmax, np.sin(dec), ra)


def synthesize(nz: int, nphi: int, lmax: int, alm: np.ndarray,
               rings_per_block: int = 8) -> np.ndarray:
    """I[nu][p] = sum_lm Y(p, lm) a(nu, lm)   (eq. fg_harmonic_matrix, forward).

    Y is evaluated a few rings at a time so that large grids fit in memory;
    each pixel's value is the plain sum over modes.
    """
    alm = np.atleast_2d(alm)
    out = np.empty((alm.shape[0], nz * nphi))
    z, alpha, _ = grid(nz, nphi)
    for j0 in range(0, nz, rings_per_block):
        j1 = min(nz, j0 + rings_per_block)
        zz = np.repeat(z[j0:j1], nphi)
        pp = np.tile(alpha, j1 - j0)
        y = real_ylm(lmax, zz, pp)
        out[:, j0 * nphi:j1 * nphi] = alm @ y.T
    return out


def synthesize_adjoint(nz: int, nphi: int, lmax: int, d_img: np.ndarray,
                       rings_per_block: int = 8) -> np.ndarray:
    """g[nu][lm] = sum_p Y(p, lm) d_img[nu][p]  (transpose of ``synthesize``)."""
    d_img = np.atleast_2d(d_img)
    out = np.zeros((d_img.shape[0], (lmax + 1) ** 2))
    z, alpha, _ = grid(nz, nphi)
    for j0 in range(0, nz, rings_per_block):
        j1 = min(nz, j0 + rings_per_block)
        zz = np.repeat(z[j0:j1], nphi)
        pp = np.tile(alpha, j1 - j0)
        y = real_ylm(lmax, zz, pp)
        out += d_img[:, j0 * nphi:j1 * nphi] @ y
    return out
