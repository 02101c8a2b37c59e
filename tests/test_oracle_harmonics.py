"""Pins of the oracle's real spherical harmonics and synthesis."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import sky


def scipy_real_ylm(lmax, z, phi):
    """Real orthonormal Y from scipy's complex sph_harm_y, removing its (-1)^m phase."""
    theta = np.arccos(z)
    out = np.empty((z.size, (lmax + 1) ** 2))
    for l in range(lmax + 1):
        c = l * l + l
        out[:, c] = special.sph_harm_y(l, 0, theta, phi).real
        for m in range(1, l + 1):
            y = special.sph_harm_y(l, m, theta, phi) * (-1) ** m
            out[:, c + m] = math.sqrt(2) * y.real
            out[:, c - m] = math.sqrt(2) * y.imag
    return out


@pytest.mark.parametrize("lmax,npts", [(20, 300), (100, 40)])
def test_real_ylm_vs_scipy(lmax, npts):
    rng = np.random.default_rng(lmax)
    z = rng.uniform(-1, 1, npts)
    phi = rng.uniform(0, 2 * math.pi, npts)
    a = sky.real_ylm(lmax, z, phi)
    b = scipy_real_ylm(lmax, z, phi)
    np.testing.assert_allclose(a, b, atol=1e-12 * max(1.0, np.abs(b).max()))


def test_low_order_closed_forms():
    z = np.linspace(-0.99, 0.99, 7)
    phi = np.linspace(0.1, 6.0, 7)
    y = sky.real_ylm(1, z, phi)
    k = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(y[:, 0], 1 / math.sqrt(4 * math.pi), rtol=1e-15)
    np.testing.assert_allclose(y[:, 2], k * z, rtol=1e-14)                                 # l=1, m=0
    np.testing.assert_allclose(y[:, 3], k * np.sqrt(1 - z * z) * np.cos(phi), rtol=1e-14)  # m=+1
    np.testing.assert_allclose(y[:, 1], k * np.sqrt(1 - z * z) * np.sin(phi), rtol=1e-14)  # m=-1


@pytest.mark.parametrize("lmax,tol", [(20, 1e-13), (100, 1e-11)])
def test_orthonormal_gauss_legendre(lmax, tol):
    """App. A (eq. sht_ortho): the quadrature of Y Y^T over the sphere is the identity.

    Gauss-Legendre in z times a uniform rule in phi is exact for band-limited
    products (degree <= 2 lmax), so the discrete Gram matrix equals I to rounding.
    """
    nz = lmax + 1
    nphi = 2 * lmax + 2
    x, wz = np.polynomial.legendre.leggauss(nz)
    phi = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    zz = np.repeat(x, nphi)
    pp = np.tile(phi, nz)
    wgt = np.repeat(wz, nphi) * (2 * math.pi / nphi)
    y = sky.real_ylm(lmax, zz, pp)
    gram = (y * wgt[:, None]).T @ y
    assert np.max(np.abs(gram - np.eye(gram.shape[0]))) < tol


def test_equal_area_gram_is_not_identity():
    """Diagnostic: on the equal-area grid the pixel sum of Y Y^T is only close to I."""
    y = sky.basis_matrix(32, 96, 20)
    gram = (4 * math.pi / (32 * 96)) * y.T @ y
    dev = np.max(np.abs(gram - np.eye(gram.shape[0])))
    assert 1e-3 < dev < 0.5


def test_synthesis_blocks_and_transpose():
    rng = np.random.default_rng(5)
    lmax, nz, nphi = 12, 16, 40
    a = rng.normal(size=(3, (lmax + 1) ** 2))
    y = sky.basis_matrix(nz, nphi, lmax)
    img = sky.synthesize(nz, nphi, lmax, a, rings_per_block=3)
    np.testing.assert_allclose(img, a @ y.T, rtol=1e-13, atol=1e-13)
    d = rng.normal(size=(3, nz * nphi))
    g = sky.synthesize_adjoint(nz, nphi, lmax, d, rings_per_block=5)
    assert abs(np.sum(d * img) - np.sum(g * a)) < 1e-12 * np.sum(np.abs(d * img))
