"""Pins of the oracle's visibilities, chi^2 and gradients (checks (a)-(e) and more)."""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_2504_07090_amd import workload as w
from oracle import model, rime, sky

C = rime.C_LIGHT


@pytest.fixture(scope="module")
def c0():
    f = model.Field(w.C0)
    d = w.draw(w.C0)
    return f, d


def test_fringe_sign_worked_example():
    """eq. rime_discrete: K = exp(-2 pi i nu b.s / c).  With b.s nu / c = 1/4 cycle, K = -i."""
    b = np.array([[1.0, 0.0, 0.0]])
    s = np.array([[[0.6, 0.0, 0.8]]])
    nu = C / (4 * 0.6)
    v = rime.vis_direct(b, s, np.array([[[2.0]]]), np.array([nu]))
    np.testing.assert_allclose(v[0, 0, 0], -2.0j, atol=1e-15)


def test_point_source_at_zenith_check_a(c0):
    """(a) A point source at zenith gives g_i conj(g_j) B(zenith) S on every baseline."""
    f, d = c0
    s_flux = 3.7
    enu = np.zeros((w.C0.n_time, 1, 3))
    enu[..., 2] = 1.0
    bz = rime.beam(enu, f.freqs, math.radians(10), 150e6)
    np.testing.assert_allclose(bz, 1.0, rtol=0, atol=0)
    v = rime.vis_direct(f.bvec, enu, s_flux * bz, f.freqs)
    m = v * f.gain_products(d.gains)[None]
    np.testing.assert_allclose(m, s_flux * f.gain_products(d.gains)[None] * np.ones_like(m),
                               rtol=1e-15)
    # gain convention m_ij = g_i conj(g_j) V_ij: g_0 = 2, g_1 = i gives -2i S
    g = np.ones((w.C0.n_freq, 16), dtype=complex)
    g[:, 0], g[:, 1] = 2.0, 1j
    assert np.allclose((v * f.gain_products(g)[None])[0, 0, 0], -2j * s_flux, atol=1e-14)


def test_hermitian_check_b(c0):
    """(b) V(-b) = conj(V(b)) with two separate direct sums."""
    f, d = c0
    img = f.sky(d.alm)
    wgt = f.d_omega * f.beam(math.radians(10), np.arange(8)) * img[None]
    vp = rime.vis_direct(f.bvec, f.enu, wgt, f.freqs)
    vm = rime.vis_direct(-f.bvec, f.enu, wgt, f.freqs)
    np.testing.assert_allclose(vm, np.conj(vp), rtol=0, atol=1e-14 * np.abs(vp).max())


@pytest.mark.parametrize("nz,nphi,tol", [(32, 96, 1e-5), (128, 384, 1e-11)])
def test_monopole_beam_integral_check_c(nz, nphi, tol):
    """(c) A monopole I0 on a zero-length baseline gives I0 * 2 pi int_0^{pi/2} B sin(theta) dtheta."""
    cfg = w.scaled(w.C0, grid_nz=nz, grid_nphi=nphi)
    f = model.Field(cfg)
    i0 = 2.5
    fw = math.radians(10)
    wgt = f.d_omega * f.beam(fw, np.arange(cfg.n_freq)) * i0
    v = rime.vis_direct(np.zeros((1, 3)), f.enu, wgt, f.freqs)[..., 0]
    for k, nu in enumerate(f.freqs):
        sig = rime.beam_sigma(np.array([nu]), fw, 150e6)[0]
        exact = i0 * 2 * math.pi * integrate.quad(
            lambda th: math.exp(-th * th / (2 * sig * sig)) * math.sin(th), 0, math.pi / 2,
            epsabs=0, epsrel=1e-13, limit=200)[0]
        assert np.all(np.abs(v[:, k].imag) == 0)
        assert np.max(np.abs(v[:, k].real - exact)) / exact < tol


def test_unique_equals_physical(c0):
    f, d = c0
    fw = math.radians(10)
    a = model.forward(f, d.alm, d.gains, fw, mode="physical")
    b = model.forward(f, d.alm, d.gains, fw, mode="unique")
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(a))


def test_matrix_form_equals_direct_sum(c0):
    """eq. rime_matrix: y = A x with an explicit design matrix per (t, nu)."""
    f, d = c0
    fw = math.radians(10)
    img = f.sky(d.alm)
    bm = f.beam(fw, np.arange(8))
    v = f.vis_nogain(img, fw, np.arange(8), "physical")
    for t in range(w.C0.n_time):
        for k in range(w.C0.n_freq):
            a = rime.design_matrix(f.bvec, f.enu[t], bm[t, k], f.freqs[k], f.d_omega)
            np.testing.assert_allclose(a @ img[k], v[t, k], rtol=0,
                                       atol=1e-13 * np.abs(v[t, k]).max())


def test_adjoint_dot_check_e(c0):
    """(e) Re<y, A x> = <x, A^T y> for the real-linear map a -> m (gains, F fixed)."""
    f, d = c0
    rng = np.random.default_rng(11)
    fw = math.radians(10)
    x = rng.normal(size=d.alm.shape)
    y = rng.normal(size=(4, 8, 120)) + 1j * rng.normal(size=(4, 8, 120))
    ax = model.forward(f, x, d.gains, fw)
    lhs = float(np.sum(y.real * ax.real + y.imag * ax.imag))
    ga, _, _ = model.adjoint(f, x, d.gains, fw, y)
    rhs = float(np.sum(x * ga))
    assert abs(lhs - rhs) / (np.linalg.norm(ax) * np.linalg.norm(y)) < 1e-12


def test_adjoint_dot_fringe_only(c0):
    """Transpose pair of the fringe sum itself (weights -> V and omega -> Z)."""
    f, _ = c0
    rng = np.random.default_rng(12)
    wgt = rng.normal(size=(4, 8, f.enu.shape[1])) * f.up[:, None, :]
    om = rng.normal(size=(4, 8, 24)) + 1j * rng.normal(size=(4, 8, 24))
    v = rime.vis_direct(f.ubl_vec, f.enu, wgt, f.freqs)
    z = rime.fringe_adjoint(f.ubl_vec, f.enu, om, f.freqs, f.up)
    lhs = float(np.sum((om * v).real))
    assert abs(lhs - float(np.sum(wgt * z))) < 1e-12 * np.linalg.norm(v) * np.linalg.norm(om)


@pytest.fixture(scope="module")
def c0_data(c0):
    f, d = c0
    m, sig, data = model.make_data(f, d)
    return f, d, sig, data


def test_chi2_at_truth(c0_data):
    """At the truth chi^2 ~ chi-square with 2 N_vis degrees of freedom (mean 2N, sd 2 sqrt(N))."""
    f, d, sig, data = c0_data
    fw = math.radians(10)
    x2 = model.chi2(f, data, sig, model.forward(f, d.alm, d.gains, fw))
    n = data.size
    assert abs(x2 - 2 * n) < 5 * 2 * math.sqrt(n)


def test_grad_alm_exact_fd(c0_data):
    """chi^2 is quadratic in a, so a central difference is exact up to rounding."""
    f, d, sig, data = c0_data
    fw = math.radians(10)
    x2, ga, gg, gf = model.chi2_and_grad(f, data, sig, d.alm, d.gains, fw)
    rng = np.random.default_rng(21)
    for _ in range(6):
        i, k = rng.integers(8), rng.integers(w.C0.n_modes)
        h = 1e-2
        ap, am = d.alm.copy(), d.alm.copy()
        ap[i, k] += h
        am[i, k] -= h
        fd = (model.chi2(f, data, sig, model.forward(f, ap, d.gains, fw))
              - model.chi2(f, data, sig, model.forward(f, am, d.gains, fw))) / (2 * h)
        assert abs(fd - ga[i, k]) <= 1e-9 * max(abs(fd), 1e-3 * abs(x2) / 1e3) + 1e-7


def test_grad_gains_and_fwhm_fd(c0_data):
    f, d, sig, data = c0_data
    fw = math.radians(10)
    x2, ga, gg, gf = model.chi2_and_grad(f, data, sig, d.alm, d.gains, fw)
    rng = np.random.default_rng(22)
    h = 1e-4 * 0.05
    for _ in range(4):
        i, k = rng.integers(8), rng.integers(16)
        for comp, ref in ((1.0, gg[i, k].real), (1j, gg[i, k].imag)):
            gp, gm = d.gains.copy(), d.gains.copy()
            gp[i, k] += h * comp
            gm[i, k] -= h * comp
            fd = (model.chi2(f, data, sig, model.forward(f, d.alm, gp, fw))
                  - model.chi2(f, data, sig, model.forward(f, d.alm, gm, fw))) / (2 * h)
            assert abs(fd - ref) <= 1e-6 * abs(ref) + 1e-6 * math.sqrt(abs(x2))
    # F enters through exp(-theta^2 / 2 sigma^2): Richardson-extrapolated central difference
    def cd(hf):
        return (model.chi2(f, data, sig, model.forward(f, d.alm, d.gains, fw + hf))
                - model.chi2(f, data, sig, model.forward(f, d.alm, d.gains, fw - hf))) / (2 * hf)
    hf = 1e-4 * fw
    fd = (4 * cd(hf / 2) - cd(hf)) / 3
    assert abs(fd - gf) <= 1e-6 * abs(gf)


def test_physical_and_unique_gradients_agree(c0_data):
    f, d, sig, data = c0_data
    fw = math.radians(10)
    a = model.chi2_and_grad(f, data, sig, d.alm, d.gains, fw, mode="physical")
    b = model.chi2_and_grad(f, data, sig, d.alm, d.gains, fw, mode="unique")
    assert abs(a[0] - b[0]) < 1e-12 * a[0]
    for x, y in zip(a[1:3], b[1:3]):
        assert np.max(np.abs(x - y)) < 1e-11 * np.max(np.abs(x))
    assert abs(a[3] - b[3]) < 1e-11 * abs(a[3])


def test_channel_subset_is_a_slice(c0_data):
    """Every term of the model is per channel: a channel subset reproduces the slice."""
    f, d, sig, data = c0_data
    fw = math.radians(10)
    full = model.forward(f, d.alm, d.gains, fw)
    sub = model.forward(f, d.alm, d.gains, fw, chans=[2, 5])
    np.testing.assert_allclose(sub, full[:, [2, 5]], rtol=0, atol=1e-14 * np.abs(full).max())


def test_single_time_field_equals_time_sample():
    """A field holding only time sample t (LST0 set to that sample's LST) gives the
    same visibilities and adjoint as sample t of the full field; the full-size
    GPU parity tests evaluate the oracle one time sample at a time this way."""
    cfg = w.scaled(w.C0, n_freq=3, lmax=8)
    f = model.Field(cfg)
    d = w.draw(cfg)
    fw = w.fwhm_ref_rad(cfg)
    full = model.forward(f, d.alm, d.gains, fw)
    rng = np.random.default_rng(3)
    y = rng.normal(size=full.shape) + 1j * rng.normal(size=full.shape)
    for t in (0, 2):
        ft = model.Field(w.scaled(cfg, n_time=1, lst0_rad=float(w.lsts(cfg)[t])))
        one = model.forward(ft, d.alm, d.gains, fw, chans=[1, 2])
        assert np.max(np.abs(one[0] - full[t, 1:3])) <= 1e-13 * np.max(np.abs(full))
    ysel = np.zeros_like(y)
    ysel[1] = y[1]
    ga, gg, gf = model.adjoint(f, d.alm, d.gains, fw, ysel)
    ft = model.Field(w.scaled(cfg, n_time=1, lst0_rad=float(w.lsts(cfg)[1])))
    ga1, gg1, gf1 = model.adjoint(ft, d.alm, d.gains, fw, y[1:2])
    assert np.max(np.abs(ga1 - ga)) <= 1e-12 * np.max(np.abs(ga))
    assert np.max(np.abs(gg1 - gg)) <= 1e-12 * np.max(np.abs(gg))
    assert abs(gf1 - gf) <= 1e-12 * abs(gf)
