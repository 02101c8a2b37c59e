"""Pins of the map-making oracle (eq. vis_to_map, eq. map_psf).

- Re(A^H y) through the explicit response matrix equals the pixel-space
  adjoint of the forward model (a separate route: the fringe transpose loop
  with unique baselines), for the same cotangent y.
- The weight sum_rows |A_rp|^2 has the closed form
  dOmega^2 sum_t B(p, t)^2 sum_{i<j} |g_i g_j|^2.
- The point-spread function is unit on its diagonal: the map of y = A e_p
  is 1 at pixel p, for any visible p.
- Pixels never above the horizon, and pixels below the weight floor, map to 0.
"""
import numpy as np

from oracle import mapmaking as mm
from oracle import model, rime
from paper_2504_07090_amd import workload as w

CFG = w.scaled(w.C0, n_freq=2, n_time=3)


def _setup():
    d = w.draw(CFG)
    of = model.Field(CFG)
    return d, of, w.fwhm_ref_rad(CFG)


def test_adjoint_routes_agree():
    d, of, fw = _setup()
    rng = np.random.default_rng(3)
    y = rng.normal(size=(CFG.n_time, CFG.n_freq, len(of.pairs))) + 1j * rng.normal(size=(CFG.n_time, CFG.n_freq, len(of.pairs)))
    # route 1: explicit matrix
    a = mm.response_matrix(of, d.gains, fw, 1)
    r1 = np.real(np.conj(a).T @ y[:, 1, :].reshape(-1))
    # route 2: the forward model's pixel-space adjoint (d_img of model.adjoint)
    gp = of.gain_products(d.gains[[1]])
    omega = np.conj(y[:, [1], :]) * gp[None]
    z = rime.fringe_adjoint(of.bvec, of.enu, omega, of.freqs[[1]], of.up)
    r2 = of.d_omega * np.sum(of.beam(fw, [1]) * z, axis=0)[0]
    assert np.max(np.abs(r1 - r2)) <= 1e-12 * np.max(np.abs(r1))


def test_weight_closed_form():
    d, of, fw = _setup()
    _, wgt = mm.dirty_map(of, np.zeros((CFG.n_time, CFG.n_freq, len(of.pairs)), complex), d.gains, fw)
    g2 = np.abs(of.gain_products(d.gains)) ** 2                          # [nf][bl]
    bm = of.beam(fw, range(CFG.n_freq))                                  # [t][nf][p]
    ref = of.d_omega ** 2 * np.sum(bm ** 2, axis=0) * np.sum(g2, axis=1)[:, None]
    assert np.max(np.abs(wgt - ref)) <= 1e-12 * np.max(ref)


def test_psf_unit_diagonal_and_invisible_pixels():
    d, of, fw = _setup()
    a = mm.response_matrix(of, d.gains, fw, 0)
    vis_pix = np.flatnonzero(np.sum(np.abs(a) ** 2, axis=0) > 0)
    rng = np.random.default_rng(4)
    wmax = np.max(np.sum(np.abs(a) ** 2, axis=0))
    good = [p for p in vis_pix if np.sum(np.abs(a[:, p]) ** 2) >= mm.WEIGHT_FLOOR * wmax]
    for p in rng.choice(good, size=5, replace=False):
        y = np.zeros((CFG.n_time, CFG.n_freq, len(of.pairs)), complex)
        y[:, 0, :] = a[:, p].reshape(CFG.n_time, -1)
        xh, _ = mm.dirty_map(of, y, d.gains, fw)
        assert abs(xh[0, p] - 1.0) <= 1e-12
    never = np.setdiff1d(np.arange(a.shape[1]), vis_pix)
    assert len(never) > 0
    y = rng.normal(size=(CFG.n_time, CFG.n_freq, len(of.pairs))) + 0j
    xh, wgt = mm.dirty_map(of, y, d.gains, fw)
    assert np.all(xh[:, never] == 0.0)
    low = wgt[0] < mm.WEIGHT_FLOOR * wgt[0].max()
    assert np.any(low & (wgt[0] > 0)) and np.all(xh[0, low] == 0.0)
