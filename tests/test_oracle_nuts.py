"""Pins of the oracle's No-U-Turn sampler (Sec. 4.2; Hoffman & Gelman 2014,
Betancourt 2017): its samples of Gaussians have the right moments, one
doubling is a one-step Metropolis HMC transition, and the termination of a
harmonic oscillator's trajectory sits near half a period."""
import math

import numpy as np
import pytest

from oracle import hmc, nuts


def _gauss(mu, cov):
    prec = np.linalg.inv(cov)
    return lambda q: (0.5 * float((q - mu) @ prec @ (q - mu)), prec @ (q - mu))


@pytest.mark.parametrize("mass", ["unit", "dense"])
def test_nuts_samples_correlated_gaussian(mass):
    """Mean and covariance of a rho = 0.9 Gaussian, with a unit mass (the
    trajectories must bend round the correlation) and with the dense mass equal
    to its precision."""
    mu = np.array([1.0, -0.5])
    cov = np.array([[1.0, 0.9], [0.9, 1.0]])
    pg = _gauss(mu, cov)
    m = np.ones(2) if mass == "unit" else hmc.BlockMass(np.ones(2), [(0, np.linalg.cholesky(np.linalg.inv(cov)))])
    q = np.zeros(2)
    u, g = pg(q)
    xs, steps = [], []
    for t in range(2500):
        r = nuts.trajectory(q, u, g, 0.25, 6, m, pg, 21, 0, t)
        q, u, g = r.q, r.u, r.g
        steps.append(r.n_steps)
        if t >= 100:
            xs.append(q.copy())
    xs = np.array(xs)
    assert np.all(np.abs(xs.mean(0) - mu) < 0.1)
    assert np.max(np.abs(np.cov(xs.T) - cov)) < 0.1
    assert max(steps) < 63    # the criterion, not the depth limit, ends trajectories


def test_one_doubling_is_one_step_metropolis():
    """With max_depth 1 the proposal is the one leapfrog step's end point, taken
    with probability min(1, exp(H0 - H1)) (the merge uniform of doubling 0)."""
    pg = _gauss(np.zeros(3), np.diag([1.0, 2.0, 0.5]))
    q0 = np.array([0.3, -1.0, 0.7])
    u0, g0 = pg(q0)
    minv = np.array([1.0, 1.5, 0.7])
    moved = 0
    for t in range(40):
        r = nuts.trajectory(q0, u0, g0, 0.9, 1, minv, pg, 4, 1, t)
        p0 = hmc.draw_momentum(minv, 4, 1, t)
        v = nuts.direction(4, 1, t, 0)
        q1, p1, u1, g1 = hmc.leapfrog(q0, p0, g0, v * 0.9, 1, minv, pg)
        h0 = u0 + hmc.kinetic(p0, minv)
        h1 = u1 + hmc.kinetic(p1, minv)
        assert r.n_steps == 1 and abs(r.h0 - h0) <= 1e-12 * abs(h0)
        take = nuts.merge_uniform(4, 1, t, 0) < math.exp(min(0.0, h0 - h1))
        assert r.moved == take
        if take:
            moved += 1
            assert np.max(np.abs(r.q - q1)) <= 1e-14 and abs(r.h_prop - h1) <= 1e-12 * abs(h1)
        else:
            assert np.array_equal(r.q, q0)
    assert 0 < moved < 40


def test_harmonic_oscillator_turns_near_half_period():
    """U = |q|^2/2 in 100 dimensions, unit mass: every coordinate oscillates with
    period 2 pi, and with many random phases the displacement over a span T is
    orthogonal to the end velocity exactly when sin T = 0, so the criterion
    fires once a trajectory spans about half a period.  Doubling checks the
    whole trajectory at 2^k - 1 steps, so it stops between pi and about 2 pi,
    long before the depth limit of 2^10 - 1 steps."""
    pg = lambda q: (0.5 * float(q @ q), q.copy())
    eps = 0.02
    rng = np.random.default_rng(3)
    for t in range(6):
        q0 = rng.normal(size=100)
        u0, g0 = pg(q0)
        r = nuts.trajectory(q0, u0, g0, eps, 10, np.ones(100), pg, 8, 0, t)
        assert r.reason in ("turn", "subtree-turn")
        span = eps * r.n_steps
        assert 0.5 * math.pi < span < 3 * math.pi, (t, r.n_steps)


def test_planted_flipped_turn_sign_is_caught(monkeypatch):
    orig = nuts.turns
    monkeypatch.setattr(nuts, "turns", lambda m, a, b, r, margins=None: not orig(m, a, b, r))
    with pytest.raises(AssertionError):
        test_harmonic_oscillator_turns_near_half_period()


def test_planted_last_leaf_candidate_is_caught(monkeypatch):
    """Taking every subtree's last leaf as its candidate (no multinomial draw)
    biases the samples."""
    monkeypatch.setattr(nuts, "leaf_uniform", lambda *a: 0.0)
    with pytest.raises(AssertionError):
        test_nuts_samples_correlated_gaussian("unit")
