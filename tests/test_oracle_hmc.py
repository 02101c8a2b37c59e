"""Pins of the oracle's Philox stream and HMC integrator."""
import json
import math
import os

import numpy as np
import pytest

from paper_2504_07090_amd import workload as w
from oracle import hmc, model, philox


def test_philox_known_answers(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "philox_kat.json")))
    for v in g["vectors"]:
        out = philox.philox4x32_10([int(x, 16) for x in v["ctr"]], [int(x, 16) for x in v["key"]])
        assert list(out) == [int(x, 16) for x in v["out"]]


def test_box_muller_moments():
    z = philox.normals(20000, seed=7, stream=3, traj=0)
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / z.size)
    z2 = philox.normals(20000, seed=7, stream=3, traj=1)
    assert abs(np.corrcoef(z, z2)[0, 1]) < 5 / math.sqrt(z.size)


def test_leapfrog_harmonic_oscillator_closed_form():
    """U = k q^2/2, unit mass: one leapfrog step is the matrix
    [[1 - e^2 k/2, e], [-e k (1 - e^2 k/4), 1 - e^2 k/2]]."""
    k, eps = 1.7, 0.3
    pg = lambda q: (0.5 * k * float(q @ q), k * q)
    q0, p0 = np.array([0.4]), np.array([-1.1])
    q1, p1, _, _ = hmc.leapfrog(q0, p0, k * q0, eps, 1, np.ones(1), pg)
    a = 1 - eps * eps * k / 2
    assert abs(q1[0] - (a * q0[0] + eps * p0[0])) < 1e-15
    assert abs(p1[0] - (-eps * k * (1 - eps * eps * k / 4) * q0[0] + a * p0[0])) < 1e-15


@pytest.fixture(scope="module")
def tiny_posterior():
    cfg = w.scaled(w.C0, lmax=2, n_freq=2, n_time=2, grid_nz=16, grid_nphi=48)
    f = model.Field(cfg)
    d = w.draw(cfg)
    _, sig, data = model.make_data(f, d)
    post = hmc.Posterior(f, data, sig, d.alm_var, cfg.gain_scatter)
    q0 = hmc.pack(d.alm, d.gains, w.fwhm_ref_rad(cfg))
    # inverse mass = 1 / diagonal Hessian, by differences of the gradient
    _, g0 = post.potential_and_grad(q0)
    hdiag = np.empty(q0.size)
    for i in range(q0.size):
        h = 1e-6 * max(1.0, abs(q0[i]))
        qp = q0.copy()
        qp[i] += h
        hdiag[i] = (post.potential_and_grad(qp)[1][i] - g0[i]) / h
    return post, q0, 1.0 / hdiag


def test_posterior_gradient_fd(tiny_posterior):
    post, q0, _ = tiny_posterior
    u0, g0 = post.potential_and_grad(q0)
    rng = np.random.default_rng(4)
    for i in rng.choice(q0.size, 6, replace=False):
        h = 1e-6 * max(1.0, abs(q0[i]))
        qp, qm = q0.copy(), q0.copy()
        qp[i] += h
        qm[i] -= h
        fd = (post.potential_and_grad(qp)[0] - post.potential_and_grad(qm)[0]) / (2 * h)
        assert abs(fd - g0[i]) < 1e-5 * max(1.0, abs(g0[i]))


def test_leapfrog_reversible_and_second_order(tiny_posterior):
    post, q0, minv = tiny_posterior
    assert np.all(minv > 0)
    u0, g0 = post.potential_and_grad(q0)
    p0 = hmc.draw_momentum(minv, seed=5, stream=0, traj=0)
    q1, p1, u1, g1 = hmc.leapfrog(q0, p0, g0, 0.1, 10, minv, post.potential_and_grad)
    q2, p2, _, _ = hmc.leapfrog(q1, -p1, g1, 0.1, 10, minv, post.potential_and_grad)
    assert np.max(np.abs(q2 - q0)) < 1e-10 * np.max(np.abs(q0))
    assert np.max(np.abs(-p2 - p0)) < 1e-8 * np.max(np.abs(p0))
    # energy error shrinks as eps^2 at fixed trajectory length
    errs = []
    for eps, n in ((0.1, 5), (0.05, 10)):
        qe, pe, ue, _ = hmc.leapfrog(q0, p0, g0, eps, n, minv, post.potential_and_grad)
        errs.append(abs((ue + hmc.kinetic(pe, minv)) - (u0 + hmc.kinetic(p0, minv))))
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_hmc_samples_gaussian():
    """HMC on a 2-D Gaussian reproduces its mean and variances (statistical)."""
    mu = np.array([1.0, -2.0])
    var = np.array([0.5, 2.0])
    pg = lambda q: (0.5 * float(np.sum((q - mu) ** 2 / var)), (q - mu) / var)
    q = np.zeros(2)
    u, g = pg(q)
    xs = []
    for t in range(3000):
        q, u, g, acc, h0, h1 = hmc.trajectory(q, u, g, 0.4, 8, np.ones(2), pg, 9, 0, t)
        if t >= 200:
            xs.append(q.copy())
    xs = np.array(xs)
    assert np.all(np.abs(xs.mean(0) - mu) < 6 * np.sqrt(var / 300))
    assert np.all(np.abs(xs.var(0) / var - 1) < 0.25)
