"""Map-making from visibilities (oracle).

Sec. 4.3 (map-making, eq. map_to_vis, eq. vis_to_map, eq. map_psf): for one
channel the visibilities are y = A x + n, with A the beam-and-fringe response
of eq. rime_matrix stacked over times and baselines (here including the
antenna gains, A[(t, ij)][p] = dOmega B(p, t) g_i conj(g_j)
exp(-2 pi i nu b_ij . s_p(t) / c)), and the map estimate is
    x_hat = D A^H N^-1 y.
For a real sky and N proportional to the identity the real part is the
estimate, and the diagonal normalisation D = diag(Re A^H N^-1 A)^-1 (the
paper uses a diagonal D) makes the point-spread function P = D A^H N^-1 A
unit on its diagonal; the noise level then cancels:
    x_hat_p = Re(A^H y)_p / sum_rows |A_rp|^2.
Reading: where the response is negligible the ratio only amplifies noise
(it grows like 1 / B), so pixels whose weight sum_rows |A_rp|^2 is below
WEIGHT_FLOOR times the channel's largest weight (beam power ~1e-6 of the
best-covered pixel) are set to 0, as are pixels never above the horizon.
"""
from __future__ import annotations

import numpy as np

from . import model, rime

WEIGHT_FLOOR = 1e-6


def response_matrix(field: model.Field, gains: np.ndarray, fwhm: float, chan: int) -> np.ndarray:
    """A [(t, ij)][p] of one channel, explicitly (eq. rime_matrix with gains)."""
    nu = field.freqs[chan]
    bm = field.beam(fwhm, [chan])[:, 0, :]                       # [t][p], zero below the horizon
    gp = field.gain_products(gains[[chan]])[0]                    # [bl]
    rows = []
    for t in range(len(field.lst)):
        a = rime.design_matrix(field.bvec, field.enu[t], bm[t], nu, field.d_omega)   # [bl][p]
        rows.append(gp[:, None] * a)
    return np.concatenate(rows, axis=0)


def dirty_map(field: model.Field, data: np.ndarray, gains: np.ndarray, fwhm: float):
    """(x_hat [n_freq][n_pix], weight [n_freq][n_pix] = sum_rows |A_rp|^2)."""
    nf = len(field.freqs)
    npix = field.enu.shape[1]
    out = np.zeros((nf, npix))
    wgt = np.zeros((nf, npix))
    for f in range(nf):
        a = response_matrix(field, gains, fwhm, f)
        y = data[:, f, :].reshape(-1)
        num = np.real(np.conj(a).T @ y)
        den = np.sum(np.abs(a) ** 2, axis=0)
        wgt[f] = den
        keep = den >= WEIGHT_FLOOR * np.max(den)
        out[f, keep] = num[keep] / den[keep]
    return out, wgt
